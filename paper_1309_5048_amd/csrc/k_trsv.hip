// Level-scheduled sparse triangular solves with the IC(0) factor (L y = r, L^T z = y),
// the latency-bound step of the velocity preconditioner (IC(0) of A, Sec. 6.4 of the
// paper).
//
// One cooperative workgroup per group of rows (a spatial strip of one velocity
// component).  Three wavefronts with separate jobs, synchronised through LDS counters:
//   wave 0 (compute): walks the group's steps (rows of one dependency level), gathers
//          dependency values from LDS slots, reduces over kTrsvG lanes per row, keeps
//          the result in its LDS slot and hands (row, value) to the writer through an
//          LDS ring.  Schedule entries, reciprocal diagonals and right-hand sides
//          (pre-gathered into schedule order) are prefetched D steps ahead into
//          registers; the wave issues no global stores and no fences.
//   wave 1 (halo):    stages values of rows owned by other groups into their LDS slots
//          once the producing group has published the level containing them
//          (agent-scope acquire) and the slot's previous occupant is dead.
//   wave 2 (writer):  drains the ring to global memory, accumulates the optional fused
//          dot product, and publishes the group's progress (agent-scope release) at
//          the levels other groups wait for.
// All waits are bounded; a timeout sets a device error flag and every wave drains, so
// the kernel always terminates.  Progress values are epoch * kLevelStride + level + 1
// with a device epoch advanced by the last workgroup, so counters need no reset.
#include "stokes_internal.h"

namespace stk {

struct TrsvArgs {
  const int32_t* grp_step_ptr;
  const int32_t* grp_halo_ptr;
  const int32_t* halo_row;
  const int32_t* halo_grp;
  const int32_t* halo_lvl;
  const int32_t* halo_slot;
  const int32_t* halo_free;
  const int32_t* step_level;
  const int32_t* step_halo_need;
  const int32_t* step_publish;
  const int32_t* srow;
  const int32_t* sslot;
  const int32_t* ent_src;
  unsigned long long* progress;
  unsigned long long* epoch;
  unsigned int* done_count;
  int* err;
  double* partials;
  int E;
  int ngroups;
  int nslots;
  int nrows;
};

constexpr long kSpinLimit = 1L << 24;

__device__ __forceinline__ int to_vgpr(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

__device__ __forceinline__ bool err_set(const int* err) {
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void raise_err(int* err) {
  __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lds_load_acq(int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store_rel(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until the LDS counter reaches `need`; returns the observed value (or `need` after
// a timeout / a raised error flag).
__device__ __forceinline__ int lds_wait(int* ctr, int need, int* err) {
  int v = lds_load_acq(ctr);
  long spins = 0;
  while (v < need) {
    if (((++spins) & 255) == 0) {
      if (spins > kSpinLimit) {
        raise_err(err);
        return need;
      }
      if (err_set(err)) return need;
    }
    v = lds_load_acq(ctr);
  }
  return v;
}

enum { CTR_COMPUTED = 0, CTR_HALO = 1, CTR_WRITTEN = 2 };

template <typename T, int R>
struct Ring {
  // one step of output: rows, values, level, publish flag
  int row[kTrsvRPS];
  T val[kTrsvRPS][R];
  int level;
  int publish;
};

template <typename T, int R, int EM, int D>
__global__ __launch_bounds__(kTrsvThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trsv(
    TrsvArgs a, const T* __restrict__ ent_val, const T* __restrict__ sdinv, const T* __restrict__ rhs_s,
    T* __restrict__ out, const T* __restrict__ dotv, double* __restrict__ dot_out, const int* __restrict__ skip) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (skip != nullptr && *skip) return;
  int* ctr = reinterpret_cast<int*>(smem);
  Ring<T, R>* ring = reinterpret_cast<Ring<T, R>*>(smem + 64);
  T* xs = reinterpret_cast<T*>(smem + 64 + sizeof(Ring<T, R>) * kTrsvRing);

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  const unsigned long long base = (*a.epoch) * (unsigned long long)kLevelStride;
  const int s0 = a.grp_step_ptr[g], s1 = a.grp_step_ptr[g + 1];
  const int nsteps = s1 - s0;
  const int h0 = a.grp_halo_ptr[g], h1 = a.grp_halo_ptr[g + 1];
  const int nhalo = h1 - h0;
  const int E = a.E;

  if (tid < 16) ctr[tid] = 0;
  if (tid < R) xs[tid] = T(0);  // slot 0: the zero slot read by padding entries
  __syncthreads();

  double dotacc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) dotacc[c] = 0.0;

  if (wid == 0) {
    // ------------------------------ compute wave ------------------------------
    const int q = lane % kTrsvG;
    const int r = lane / kTrsvG;
    T pv[D][EM];
    int ps[D][EM];
    int pslot[D], pneed[D], prow[D], plev[D], ppub[D];
    T pdinv[D];
    T prhs[D][R];
    int halo_seen = 0, written_seen = 0;
    auto load = [&](int d, int ss) {
      const int v_ss = to_vgpr(ss);
#pragma unroll
      for (int e = 0; e < EM; ++e) {
        if (e < E) {
          const size_t off = ((size_t)v_ss * E + e) * 64 + lane;
          pv[d][e] = ent_val[off];
          ps[d][e] = a.ent_src[off];
        } else {
          pv[d][e] = T(0);
          ps[d][e] = 0;
        }
      }
      const size_t ro = (size_t)v_ss * kTrsvRPS + r;
      pslot[d] = a.sslot[ro];
      prow[d] = a.srow[ro];
      pdinv[d] = sdinv[ro];
#pragma unroll
      for (int c = 0; c < R; ++c) prhs[d][c] = rhs_s[ro * R + c];
      pneed[d] = a.step_halo_need[v_ss];
      plev[d] = a.step_level[v_ss];
      ppub[d] = a.step_publish[v_ss];
    };
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (s0 + d < s1) load(d, s0 + d);
    for (int s = s0; s < s1; s += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int ss = s + d;
        if (ss < s1) {
          const int k = ss - s0;
          if (pneed[d] > halo_seen) halo_seen = lds_wait(&ctr[CTR_HALO], pneed[d], a.err);
          if (k - kTrsvRing + 1 > written_seen) written_seen = lds_wait(&ctr[CTR_WRITTEN], k - kTrsvRing + 1, a.err);
          T acc[R];
#pragma unroll
          for (int c = 0; c < R; ++c) acc[c] = T(0);
#pragma unroll
          for (int e = 0; e < EM; ++e) {
            const T v = pv[d][e];
            const T* xp = xs + (size_t)ps[d][e] * R;
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] = fma(v, xp[c], acc[c]);
          }
#pragma unroll
          for (int off = kTrsvG / 2; off >= 1; off >>= 1)
#pragma unroll
            for (int c = 0; c < R; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
          Ring<T, R>& rg = ring[k % kTrsvRing];
          if (q == 0) {
            const int slot = pslot[d];
            T res[R];
#pragma unroll
            for (int c = 0; c < R; ++c) res[c] = (prhs[d][c] - acc[c]) * pdinv[d];
            if (slot > 0) {
              T* xp = xs + (size_t)slot * R;
#pragma unroll
              for (int c = 0; c < R; ++c) xp[c] = res[c];
            }
            rg.row[r] = prow[d];
#pragma unroll
            for (int c = 0; c < R; ++c) rg.val[r][c] = res[c];
          }
          if (lane == 0) {
            rg.level = plev[d];
            rg.publish = ppub[d];
            lds_store_rel(&ctr[CTR_COMPUTED], k + 1);
          }
          if (ss + D < s1) load(d, ss + D);
        }
      }
    }
  } else if (wid == 1) {
    // ------------------------------- halo wave --------------------------------
    int pos = 0;
    long spins = 0;
    while (pos < nhalo) {
      const int idx = pos + lane;
      const bool valid = idx < nhalo;
      int grp = 0, lvl = 0, row = 0, slot = 0, fr = 0;
      if (valid) {
        grp = a.halo_grp[h0 + idx];
        lvl = a.halo_lvl[h0 + idx];
        row = a.halo_row[h0 + idx];
        slot = a.halo_slot[h0 + idx];
        fr = a.halo_free[h0 + idx];
      }
      bool ready = true;
      if (valid) {
        const int comp = lds_load_acq(&ctr[CTR_COMPUTED]);
        const unsigned long long p = __hip_atomic_load(a.progress + grp, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        ready = (comp >= fr) && (p >= base + (unsigned long long)lvl + 1ull);
      }
      const unsigned long long notready = __ballot(!ready);
      int count = notready ? __ffsll((long long)notready) - 1 : 64;
      count = min(count, nhalo - pos);
      if (count == 0) {
        ++spins;
        if ((spins & 63) == 0 && (spins > (kSpinLimit >> 6) || err_set(a.err))) {
          if (spins > (kSpinLimit >> 6)) raise_err(a.err);
          if (lane == 0) lds_store_rel(&ctr[CTR_HALO], nhalo);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      if (lane < count && row >= 0 && row < a.nrows && slot > 0 && slot < a.nslots) {
        T* xp = xs + (size_t)slot * R;
#pragma unroll
        for (int c = 0; c < R; ++c) xp[c] = out[(size_t)row * R + c];
      }
      pos += count;
      if (lane == 0) lds_store_rel(&ctr[CTR_HALO], pos);
    }
  } else {
    // ------------------------------ writer wave -------------------------------
    int written = 0;
    while (written < nsteps) {
      const int avail = min(nsteps, lds_wait(&ctr[CTR_COMPUTED], written + 1, a.err));
      int maxpub = -1;
      for (int k0 = written; k0 < avail; k0 += 64 / kTrsvRPS) {
        const int k = k0 + lane / kTrsvRPS;
        const int r = lane % kTrsvRPS;
        int row = -1;
        T v[R];
        if (k < avail) {
          const Ring<T, R>& rg = ring[k % kTrsvRing];
          row = rg.row[r];
#pragma unroll
          for (int c = 0; c < R; ++c) v[c] = rg.val[r][c];
          if (r == 0 && rg.publish) maxpub = max(maxpub, rg.level);
        }
        if (k0 + 64 / kTrsvRPS >= avail && lane == 0) lds_store_rel(&ctr[CTR_WRITTEN], avail);
        if (row >= 0 && row < a.nrows) {
#pragma unroll
          for (int c = 0; c < R; ++c) out[(size_t)row * R + c] = v[c];
          if (dotv != nullptr) {
#pragma unroll
            for (int c = 0; c < R; ++c) dotacc[c] += (double)v[c] * (double)dotv[(size_t)row * R + c];
          }
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) maxpub = max(maxpub, __shfl_xor(maxpub, off, 64));
      if (maxpub >= 0 && lane == 0)
        __hip_atomic_store(a.progress + g, base + (unsigned long long)maxpub + 1ull, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
      written = avail;
    }
  }
  __syncthreads();

  // ----------------------- epilogue: fused dot and epoch -----------------------
  if (dotv != nullptr && wid == 2) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double v = dotacc[c];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) a.partials[(size_t)g * R + c] = v;
    }
  }
  __syncthreads();
  if (tid == 128) {
    __threadfence();
    const unsigned int prev = __hip_atomic_fetch_add(a.done_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == (unsigned int)(a.ngroups - 1)) {
      __threadfence();
      if (dotv != nullptr) {
        for (int c = 0; c < R; ++c) {
          double v = 0.0;
          for (int k = 0; k < a.ngroups; ++k)
            v += __hip_atomic_load(a.partials + (size_t)k * R + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          dot_out[c] = v;
        }
      }
      __hip_atomic_store(a.done_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.epoch, *a.epoch + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// rhs gathered into schedule order: rhs_s[(step*RPS + r)*R + c] = rhs[row*R + c]
template <typename T, int R>
__global__ void k_trsv_gather_rhs(int64_t nslots_rows, const int32_t* __restrict__ srow, const T* __restrict__ rhs,
                                  T* __restrict__ rhs_s, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nslots_rows * R;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / R;
    const int c = int(t % R);
    const int row = srow[k];
    rhs_s[t] = row >= 0 ? rhs[(size_t)row * R + c] : T(0);
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename T, int R>
size_t trsv_shmem_t(int nslots) {
  return 64 + sizeof(Ring<T, R>) * kTrsvRing + (size_t)nslots * R * sizeof(T);
}

size_t trsv_shmem_bytes(int nslots, bool fp32, int R) {
  if (fp32) {
    switch (R) {
      case 1: return trsv_shmem_t<float, 1>(nslots);
      case 8: return trsv_shmem_t<float, 8>(nslots);
      default: return trsv_shmem_t<float, 16>(nslots);
    }
  }
  switch (R) {
    case 1: return trsv_shmem_t<double, 1>(nslots);
    case 8: return trsv_shmem_t<double, 8>(nslots);
    default: return trsv_shmem_t<double, 16>(nslots);
  }
}

template <typename T, int R, int EM, int D>
static hipError_t launch_trsv_t(const TrsvSchedDev& S, const T* ent_val, const T* sdinv, const T* rhs, T* out,
                                const T* dotv, double* dot_out, const int* skip, hipStream_t st) {
  TrsvArgs a;
  a.grp_step_ptr = S.grp_step_ptr;
  a.grp_halo_ptr = S.grp_halo_ptr;
  a.halo_row = S.halo_row;
  a.halo_grp = S.halo_grp;
  a.halo_lvl = S.halo_lvl;
  a.halo_slot = S.halo_slot;
  a.halo_free = S.halo_free;
  a.step_level = S.step_level;
  a.step_halo_need = S.step_halo_need;
  a.step_publish = S.step_publish;
  a.srow = S.srow;
  a.sslot = S.sslot;
  a.ent_src = S.ent_src;
  a.progress = S.progress;
  a.epoch = S.epoch;
  a.done_count = S.done_count;
  a.err = S.err;
  a.partials = S.partials;
  a.E = S.E;
  a.ngroups = S.ngroups;
  a.nslots = S.nslots;
  a.nrows = S.nrows;
  T* rhs_s = reinterpret_cast<T*>(S.rhs_s);
  const int64_t nrow_slots = (int64_t)S.nsteps * kTrsvRPS;
  hipLaunchKernelGGL((k_trsv_gather_rhs<T, R>), dim3(1024), dim3(256), 0, st, nrow_slots, S.srow, rhs, rhs_s, skip);
  const size_t shmem = trsv_shmem_t<T, R>(S.nslots);
  auto fn = k_trsv<T, R, EM, D>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const T* rhs_sc = rhs_s;
  void* args[] = {&a, &ent_val, &sdinv, &rhs_sc, &out, &dotv, &dot_out, &skip};
  return hipLaunchCooperativeKernel((const void*)fn, dim3(S.ngroups), dim3(kTrsvThreads), args, (unsigned)shmem, st);
}

template <typename T, int R>
static hipError_t launch_trsv_r(const TrsvSchedDev& S, const T* ent_val, const T* sdinv, const T* rhs, T* out,
                                const T* dotv, double* dot_out, const int* skip, hipStream_t st) {
  if (S.E <= 4) return launch_trsv_t<T, R, 4, 8>(S, ent_val, sdinv, rhs, out, dotv, dot_out, skip, st);
  if (S.E <= 8) return launch_trsv_t<T, R, 8, 6>(S, ent_val, sdinv, rhs, out, dotv, dot_out, skip, st);
  return launch_trsv_t<T, R, 16, 3>(S, ent_val, sdinv, rhs, out, dotv, dot_out, skip, st);
}

hipError_t launch_trsv(const TrsvSchedDev& S, bool fp32, int R, const void* rhs, void* out, const void* dotv,
                       double* dot_out, const int* skip, hipStream_t st) {
  if (fp32) {
    const float* v = S.ent_val32;
    const float* d = S.sdinv32;
    switch (R) {
      case 1: return launch_trsv_r<float, 1>(S, v, d, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st);
      case 8: return launch_trsv_r<float, 8>(S, v, d, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st);
      case 16: return launch_trsv_r<float, 16>(S, v, d, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st);
    }
  } else {
    const double* v = S.ent_val;
    const double* d = S.sdinv;
    switch (R) {
      case 1: return launch_trsv_r<double, 1>(S, v, d, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st);
      case 8: return launch_trsv_r<double, 8>(S, v, d, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st);
      case 16: return launch_trsv_r<double, 16>(S, v, d, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st);
    }
  }
  return hipErrorInvalidValue;
}

// Gather the factor values into schedule order (and reciprocal diagonals).
__global__ void k_trsv_gather(const int64_t* __restrict__ perm, int64_t n, const double* __restrict__ Lval,
                              double* __restrict__ out, float* __restrict__ out32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[i];
    const double v = p >= 0 ? Lval[p] : 0.0;
    out[i] = v;
    if (out32) out32[i] = (float)v;
  }
}

__global__ void k_trsv_gather_dinv(const int64_t* __restrict__ dsrc, int64_t n, const double* __restrict__ Lval,
                                   double* __restrict__ out, float* __restrict__ out32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = dsrc[i];
    const double v = p >= 0 ? 1.0 / Lval[p] : 0.0;
    out[i] = v;
    if (out32) out32[i] = p >= 0 ? 1.0f / (float)Lval[p] : 0.0f;
  }
}

hipError_t launch_trsv_gather(const TrsvSchedDev& S, const double* Lval, hipStream_t st) {
  const int64_t ne = (int64_t)S.nsteps * S.E * 64;
  const int64_t nd = (int64_t)S.nsteps * kTrsvRPS;
  hipLaunchKernelGGL(k_trsv_gather, dim3(1024), dim3(256), 0, st, S.ent_perm, ne, Lval, S.ent_val, S.ent_val32);
  hipLaunchKernelGGL(k_trsv_gather_dinv, dim3(256), dim3(256), 0, st, S.sdiag_src, nd, Lval, S.sdinv, S.sdinv32);
  return hipGetLastError();
}

}  // namespace stk

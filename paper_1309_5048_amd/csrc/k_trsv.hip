// Level-scheduled sparse triangular solves with the IC(0) factor (L y = r, L^T z = y),
// the latency-bound step of the velocity preconditioner (IC(0) of A, Sec. 6.4 of the
// paper).
//
// One cooperative workgroup per group of rows (a spatial strip of one velocity
// component).  Three wavefronts with separate jobs, synchronised through LDS counters:
//   wave 0 (compute): walks the group's steps (rows of one dependency level), gathers
//          dependency values from LDS slots, reduces over kTrsvG lanes per row with DPP,
//          keeps the result in its LDS slot and hands the values to the writer through
//          an LDS ring.  The per-step records (factor values, 16-bit slot ids, row
//          records, right-hand sides pre-gathered into schedule order) are prefetched D
//          steps ahead with vector loads; the wave issues no global stores and no fences.
//   wave 1 (halo):    stages values of rows owned by other groups into their LDS slots
//          once the producing group has published the level containing them and the
//          slot's previous occupant is dead.
//   wave 2 (writer):  drains the ring to global memory, accumulates the optional fused
//          dot product, and publishes the group's progress at the levels other groups
//          wait for.
// Cross-group traffic (solution values and progress counters) uses device-scope relaxed
// loads and stores, which are coherent across the XCDs' L2 caches by themselves; the
// writer waits for its value stores to be acknowledged (vmcnt 0) before it stores the
// progress counter, and the halo wave loads values only after it has seen the counter.
// No L2 write-back or invalidation is needed on this path.
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
  const int32_t* srow;
  const uint16_t* ssrc;
  const TrsvStep* sstep;
  unsigned long long* progress;
  unsigned long long* epoch;
  unsigned int* done_count;
  int* err;
  double* partials;
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

// Device-scope (all XCDs) relaxed value transfer, on the 64/32-bit patterns.
__device__ __forceinline__ void dev_store(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), __builtin_bit_cast(unsigned long long, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dev_store(float* p, float v) {
  __hip_atomic_store(reinterpret_cast<unsigned int*>(p), __builtin_bit_cast(unsigned int, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double dev_load(const double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ float dev_load(const float* p) {
  return __builtin_bit_cast(float, __hip_atomic_load(reinterpret_cast<const unsigned int*>(p), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
}

// Wait until every vector memory operation of this wave has completed (stores acknowledged).
__device__ __forceinline__ void wait_vm_stores() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

__device__ __forceinline__ int lds_load_acq(int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_store_rel(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until the LDS counter reaches `need`; returns the observed value (or `need` after
// a timeout / a raised error flag).  Idle waves sleep between polls.
template <bool kIdle>
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
    if (kIdle) __builtin_amdgcn_s_sleep(1);
    v = lds_load_acq(ctr);
  }
  return v;
}

// Sum over the 8 lanes of an aligned lane octet with three DPP moves (xor 1 and xor 2
// inside a quad, then the mirror inside a half row), on the 32-bit halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  const int r = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(float, r);
}

template <typename T>
__device__ __forceinline__ T octet_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  return v;
}

enum { CTR_COMPUTED = 0, CTR_HALO = 1, CTR_WRITTEN = 2 };

template <typename T, int R>
struct Ring {
  T val[kTrsvRPS][R];  // one step of output values
};

template <int R>
struct RingSize {
  static constexpr int value = R == 1 ? 64 : 16;
};

template <typename T>
struct RowRec;
template <>
struct RowRec<double> {
  using type = TrsvRow64;
};
template <>
struct RowRec<float> {
  using type = TrsvRow32;
};

// 16-byte vector type of T
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};

template <typename T, int R, int EP, int D>
__global__ __launch_bounds__(kTrsvThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trsv(
    TrsvArgs a, const T* __restrict__ sval, const typename RowRec<T>::type* __restrict__ srinfo,
    const T* __restrict__ rhs_s, T* __restrict__ out, const T* __restrict__ dotv, double* __restrict__ dot_out,
    const int* __restrict__ skip) {
  constexpr int RING = RingSize<R>::value;
  constexpr int ES = (EP + 7) / 8 * 8;
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int NV = EP / VN;  // vector loads of factor values per lane and step
  extern __shared__ __align__(16) unsigned char smem[];
  if (skip != nullptr && *skip) return;
  int* ctr = reinterpret_cast<int*>(smem);
  Ring<T, R>* ring = reinterpret_cast<Ring<T, R>*>(smem + 64);
  T* xs = reinterpret_cast<T*>(smem + 64 + sizeof(Ring<T, R>) * RING);

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  const unsigned long long base = (*a.epoch) * (unsigned long long)kLevelStride;
  const int s0 = a.grp_step_ptr[g], s1 = a.grp_step_ptr[g + 1];
  const int nsteps = s1 - s0;
  const int h0 = a.grp_halo_ptr[g], h1 = a.grp_halo_ptr[g + 1];
  const int nhalo = h1 - h0;

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
    V pv[D][NV];
    uint4 ps[D][ES / 8];
    typename RowRec<T>::type pri[D];
    T prhs[D][R];
    int halo_seen = 0, written_seen = 0;
    auto load = [&](int d, int ss) {
      const int v_ss = to_vgpr(ss);
      const V* vp = reinterpret_cast<const V*>(sval + ((size_t)v_ss * 64 + lane) * EP);
#pragma unroll
      for (int k = 0; k < NV; ++k) pv[d][k] = vp[k];
      const uint4* sp = reinterpret_cast<const uint4*>(a.ssrc + ((size_t)v_ss * 64 + lane) * ES);
#pragma unroll
      for (int k = 0; k < ES / 8; ++k) ps[d][k] = sp[k];
      const size_t ro = (size_t)v_ss * kTrsvRPS + r;
      pri[d] = srinfo[ro];
#pragma unroll
      for (int c = 0; c < R; ++c) prhs[d][c] = rhs_s[ro * R + c];
    };
    // Loads are issued unconditionally (index clamped to the last step): the number of
    // loads in flight after each buffer's loads is then the same on every path, so the
    // compiler's vmcnt waits hold back only the buffer about to be used, not the whole
    // prefetch window.
    if (nsteps > 0) {
#pragma unroll
      for (int d = 0; d < D; ++d) load(d, min(s0 + d, s1 - 1));
    }
    for (int s = s0; s < s1; s += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int ss = s + d;
        if (ss < s1) {
          const int k = ss - s0;
          if (pri[d].need > halo_seen) halo_seen = lds_wait<false>(&ctr[CTR_HALO], pri[d].need, a.err);
          if (k - RING + 1 > written_seen) written_seen = lds_wait<false>(&ctr[CTR_WRITTEN], k - RING + 1, a.err);
          // two interleaved FMA chains (even / odd entries) halve the dependency latency
          T acc[R], acc2[R];
#pragma unroll
          for (int c = 0; c < R; ++c) acc[c] = acc2[c] = T(0);
#pragma unroll
          for (int e = 0; e < EP; ++e) {
            const T v = reinterpret_cast<const T*>(&pv[d][e / VN])[e % VN];
            const unsigned word = reinterpret_cast<const unsigned*>(&ps[d][e / 8])[(e % 8) / 2];
            const int src = (e & 1) ? int(word >> 16) : int(word & 0xffffu);
            const T* xp = xs + (size_t)src * R;
            if (e & 1) {
#pragma unroll
              for (int c = 0; c < R; ++c) acc2[c] = fma(v, xp[c], acc2[c]);
            } else {
#pragma unroll
              for (int c = 0; c < R; ++c) acc[c] = fma(v, xp[c], acc[c]);
            }
          }
#pragma unroll
          for (int c = 0; c < R; ++c) acc[c] = octet_sum(acc[c] + acc2[c]);
          Ring<T, R>& rg = ring[k % RING];
          if (q == 0) {
            const int slot = pri[d].slot;
            T res[R];
#pragma unroll
            for (int c = 0; c < R; ++c) res[c] = (prhs[d][c] - acc[c]) * pri[d].dinv;
            if (slot > 0) {
              T* xp = xs + (size_t)slot * R;
#pragma unroll
              for (int c = 0; c < R; ++c) xp[c] = res[c];
            }
#pragma unroll
            for (int c = 0; c < R; ++c) rg.val[r][c] = res[c];
          }
          if (lane == 0) lds_store_rel(&ctr[CTR_COMPUTED], k + 1);
        }
        load(d, min(ss + D, s1 - 1));
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
        const unsigned long long p = __hip_atomic_load(a.progress + grp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
      // values are loaded only after their producers' counters were seen (device scope)
      asm volatile("" ::: "memory");
      if (lane < count && row >= 0 && row < a.nrows && slot > 0 && slot < a.nslots) {
        T* xp = xs + (size_t)slot * R;
        T v[R];
#pragma unroll
        for (int c = 0; c < R; ++c) v[c] = dev_load(out + (size_t)row * R + c);
#pragma unroll
        for (int c = 0; c < R; ++c) xp[c] = v[c];
      }
      pos += count;
      if (lane == 0) lds_store_rel(&ctr[CTR_HALO], pos);
    }
  } else {
    // ------------------------------ writer wave -------------------------------
    // Batches of up to 64 / RPS steps: lane (k, r) handles row r of step written + k.  The
    // batch's rows and step records are loaded before the wait for the compute wave.
    constexpr int kBatch = 64 / kTrsvRPS;
    const int kk = lane / kTrsvRPS;
    const int r = lane % kTrsvRPS;
    int written = 0;
    while (written < nsteps) {
      const int k = written + kk;
      int row = -1, level = -1;
      if (k < nsteps) {
        row = a.srow[(size_t)(s0 + k) * kTrsvRPS + r];
        const int2 lp = *reinterpret_cast<const int2*>(a.sstep + s0 + k);  // level, publish
        level = lp.y ? lp.x : -1;  // publish flag set: this step ends a level others wait for
      }
      const int avail = min(min(nsteps, written + kBatch), lds_wait<true>(&ctr[CTR_COMPUTED], written + 1, a.err));
      T v[R];
      const bool mine = k < avail;
      if (mine) {
        const Ring<T, R>& rg = ring[k % RING];
#pragma unroll
        for (int c = 0; c < R; ++c) v[c] = rg.val[r][c];
      }
      if (lane == 0) lds_store_rel(&ctr[CTR_WRITTEN], avail);  // after the ring reads (release)
      if (mine && row >= 0 && row < a.nrows) {
#pragma unroll
        for (int c = 0; c < R; ++c) dev_store(out + (size_t)row * R + c, v[c]);
        if (dotv != nullptr) {
#pragma unroll
          for (int c = 0; c < R; ++c) dotacc[c] += (double)v[c] * (double)dotv[(size_t)row * R + c];
        }
      }
      int maxpub = (mine && r == 0) ? level : -1;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) maxpub = max(maxpub, __shfl_xor(maxpub, off, 64));
      if (maxpub >= 0) {
        wait_vm_stores();  // the values of the published levels are visible device-wide
        if (lane == 0)
          __hip_atomic_store(a.progress + g, base + (unsigned long long)maxpub + 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
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
  return 64 + sizeof(Ring<T, R>) * RingSize<R>::value + (size_t)nslots * R * sizeof(T);
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

template <typename T, int R, int EP, int D>
static hipError_t launch_trsv_t(const TrsvSchedDev& S, const T* sval, const typename RowRec<T>::type* srinfo,
                                const T* rhs, T* out, const T* dotv, double* dot_out, const int* skip, hipStream_t st,
                                const TrsvTiming* tm) {
  TrsvArgs a;
  a.grp_step_ptr = S.grp_step_ptr;
  a.grp_halo_ptr = S.grp_halo_ptr;
  a.halo_row = S.halo_row;
  a.halo_grp = S.halo_grp;
  a.halo_lvl = S.halo_lvl;
  a.halo_slot = S.halo_slot;
  a.halo_free = S.halo_free;
  a.srow = S.srow;
  a.ssrc = S.ssrc;
  a.sstep = S.sstep;
  a.progress = S.progress;
  a.epoch = S.epoch;
  a.done_count = S.done_count;
  a.err = S.err;
  a.partials = S.partials;
  a.ngroups = S.ngroups;
  a.nslots = S.nslots;
  a.nrows = S.nrows;
  T* rhs_s = reinterpret_cast<T*>(S.rhs_s);
  const int64_t nrow_slots = (int64_t)S.nsteps * kTrsvRPS;
  hipLaunchKernelGGL((k_trsv_gather_rhs<T, R>), dim3(1024), dim3(256), 0, st, nrow_slots, S.srow, rhs, rhs_s, skip);
  const size_t shmem = trsv_shmem_t<T, R>(S.nslots);
  auto fn = k_trsv<T, R, EP, D>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const T* rhs_sc = rhs_s;
  void* args[] = {&a, &sval, &srinfo, &rhs_sc, &out, &dotv, &dot_out, &skip};
  if (tm && tm->before) (void)hipEventRecord(tm->before, st);
  e = hipLaunchCooperativeKernel((const void*)fn, dim3(S.ngroups), dim3(kTrsvThreads), args, (unsigned)shmem, st);
  if (tm && tm->after) (void)hipEventRecord(tm->after, st);
  return e;
}

template <typename T, int R>
static hipError_t launch_trsv_r(const TrsvSchedDev& S, const T* sval, const typename RowRec<T>::type* srinfo,
                                const T* rhs, T* out, const T* dotv, double* dot_out, const int* skip, hipStream_t st,
                                const TrsvTiming* tm) {
  switch (S.EP) {
    case 4: return launch_trsv_t<T, R, 4, 8>(S, sval, srinfo, rhs, out, dotv, dot_out, skip, st, tm);
    case 8: return launch_trsv_t<T, R, 8, 6>(S, sval, srinfo, rhs, out, dotv, dot_out, skip, st, tm);
    case 12: return launch_trsv_t<T, R, 12, 4>(S, sval, srinfo, rhs, out, dotv, dot_out, skip, st, tm);
    case 16: return launch_trsv_t<T, R, 16, 3>(S, sval, srinfo, rhs, out, dotv, dot_out, skip, st, tm);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_trsv(const TrsvSchedDev& S, bool fp32, int R, const void* rhs, void* out, const void* dotv,
                       double* dot_out, const int* skip, hipStream_t st, const TrsvTiming* tm) {
  if (fp32) {
    const float* v = S.sval32;
    const TrsvRow32* ri = S.srinfo32;
    switch (R) {
      case 1: return launch_trsv_r<float, 1>(S, v, ri, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st, tm);
      case 8: return launch_trsv_r<float, 8>(S, v, ri, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st, tm);
      case 16: return launch_trsv_r<float, 16>(S, v, ri, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st, tm);
    }
  } else {
    const double* v = S.sval;
    const TrsvRow64* ri = S.srinfo;
    switch (R) {
      case 1: return launch_trsv_r<double, 1>(S, v, ri, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st, tm);
      case 8: return launch_trsv_r<double, 8>(S, v, ri, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st, tm);
      case 16: return launch_trsv_r<double, 16>(S, v, ri, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st, tm);
    }
  }
  return hipErrorInvalidValue;
}

// Factor values into schedule order and reciprocal diagonals into the row records.
__global__ void k_trsv_gather(const int64_t* __restrict__ perm, int64_t n, const double* __restrict__ Lval,
                              double* __restrict__ out, float* __restrict__ out32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[i];
    const double v = p >= 0 ? Lval[p] : 0.0;
    out[i] = v;
    out32[i] = (float)v;
  }
}

__global__ void k_trsv_gather_dinv(const int64_t* __restrict__ dsrc, int64_t n, const double* __restrict__ Lval,
                                   TrsvRow64* __restrict__ ri, TrsvRow32* __restrict__ ri32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = dsrc[i];
    ri[i].dinv = p >= 0 ? 1.0 / Lval[p] : 0.0;
    ri32[i].dinv = p >= 0 ? 1.0f / (float)Lval[p] : 0.0f;
  }
}

hipError_t launch_trsv_gather(const TrsvSchedDev& S, const double* Lval, hipStream_t st) {
  const int64_t ne = (int64_t)S.nsteps * 64 * S.EP;
  const int64_t nd = (int64_t)S.nsteps * kTrsvRPS;
  hipLaunchKernelGGL(k_trsv_gather, dim3(1024), dim3(256), 0, st, S.vperm, ne, Lval, S.sval, S.sval32);
  hipLaunchKernelGGL(k_trsv_gather_dinv, dim3(256), dim3(256), 0, st, S.dsrc, nd, Lval, S.srinfo, S.srinfo32);
  return hipGetLastError();
}

}  // namespace stk

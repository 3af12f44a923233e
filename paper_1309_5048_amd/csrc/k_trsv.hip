// Level-scheduled sparse triangular solves with the IC(0) factor (L y = r, L^T z = y),
// the latency-bound step of the velocity preconditioner (IC(0) of A, Sec. 6.4 of the
// paper).
//
// One workgroup per group of rows (a spatial strip of one velocity component); all
// groups are resident at once.  Two wavefronts with separate jobs, synchronised through LDS counters:
//   wave 0 (compute): walks the group's steps (rows of one dependency level), gathers
//          dependency values from LDS slots, reduces over kTrsvG lanes per row with DPP,
//          keeps the result in its LDS slot and stores it to global memory (device
//          scope), accumulating the optional fused dot product.  The per-step records
//          (factor values, LDS slot ids, row records, rows, right-hand side and
//          dot-vector entries gathered into schedule order) are prefetched several steps
//          ahead into registers.
//   wave 1 (halo):    stages values of rows owned by other groups into their LDS slots
//          as soon as they appear in global memory and the slot's previous occupant is
//          dead.
// Cross-group values need no counters: before each solve every output row holds a
// signalling-NaN sentinel, which no arithmetic result can equal; the halo wave polls a
// row with device-scope loads until the sentinel is gone, and the producer's
// device-scope store makes the value visible across the XCDs' L2 caches.  LDS counters
// are plain relaxed stores after the data they announce: LDS executes one workgroup's
// operations in issue order.
// All waits are bounded; a timeout sets an error flag and every wave drains, so the
// kernel always terminates.
#include "stokes_internal.h"

namespace stk {

struct TrsvArgs {
  const int32_t* grp_step_ptr;
  const int32_t* grp_ep;    // entries per lane of each group's steps (4 or the schedule's EP)
  const int64_t* grp_eoff;  // offset of each group's first step entries
  const int32_t* grp_halo_ptr;
  const int32_t* halo_row;
  const int32_t* halo_slot;
  const int32_t* halo_free;
  const int32_t* srow;
  const uint32_t* ssrc;
  unsigned int* done_count;
  int* err;
  double* partials;
  int ngroups;
  int nslots;
  int nrows;
  int ld;  // row stride of out (the full batch width; R columns are solved per launch)
  void* cpl;  // coupling rows' values (rows nrows .., same stride and column offset as out)
  int ncpl;
  int64_t nrow_slots;  // steps x kTrsvRPS: one column block's share of the gathered {rhs, dot} pairs
};

// Output sentinel (signalling NaN) and its test, on the bit patterns.
template <typename T>
struct Sentinel;
template <>
struct Sentinel<double> {
  using U = unsigned long long;
  static constexpr U bits = 0x7FF4DEADBEEF5A5AULL;
};
template <>
struct Sentinel<float> {
  using U = unsigned int;
  static constexpr U bits = 0x7FA5DEADU;
};
template <typename T>
__device__ __forceinline__ T sentinel_value() {
  return __builtin_bit_cast(T, Sentinel<T>::bits);
}
template <typename T>
__device__ __forceinline__ bool is_sentinel(T v) {
  return __builtin_bit_cast(typename Sentinel<T>::U, v) == Sentinel<T>::bits;
}

constexpr long kSpinLimit = 1L << 24;

__device__ __forceinline__ bool err_set(const int* err) {
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void raise_err(int* err) {
  __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lds_load(int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Counter store after the data it announces (compiler ordering only; see the header).
__device__ __forceinline__ void lds_signal(int* p, int v) {
  asm volatile("" ::: "memory");
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until the LDS counter reaches `need`; returns the observed value (or `need` after
// a timeout or once an error is flagged).  Errors are flagged in LDS (lerr) and, by waves
// with kGlobal, also in the device error word; the compute wave uses kGlobal = false so
// that it issues no global memory operation at all.  Idle waves sleep between polls.
template <bool kIdle, bool kGlobal>
__device__ __forceinline__ int lds_wait(int* ctr, int need, int* lerr, int* err) {
  int v = lds_load(ctr);
  long spins = 0;
  while (v < need) {
    if (((++spins) & 255) == 0) {
      if (spins > kSpinLimit) {
        lds_signal(lerr, 1);
        if (kGlobal) raise_err(err);
        return need;
      }
      if (lds_load(lerr) != 0) return need;
      if (kGlobal && err_set(err)) return need;
    }
    if (kIdle) __builtin_amdgcn_s_sleep(1);
    v = lds_load(ctr);
  }
  asm volatile("" ::: "memory");
  return v;
}

// Sum over the 8 lanes of an aligned lane octet with three DPP moves (xor 1 and xor 2
// inside a quad, then the mirror inside a half row), on the 32-bit halves of a double.
// Every source lane of these patterns lies inside the octet, so the moves need no "old"
// value.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
  const long long r = ((long long)(unsigned)lo) | ((long long)hi << 32);
  return __builtin_bit_cast(double, r);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  const int r = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(float, r);
}

template <typename T>
__device__ __forceinline__ T octet_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  return v;
}

// Octet reduce-scatter of RC (1, 2, 4 or 8) columns: v[c] holds each lane's partial of
// column c; lane q of the octet returns the octet's total of column octet_col<RC>(q).
// Each stage halves the columns a lane keeps: lane and partner (mirror inside the half row,
// then xor 2, then xor 1) keep opposite halves and add what the partner sends; once one
// column is left the remaining stages are plain all-reduce steps.  8 / RC lanes end with
// each column.
template <int RC>
__device__ __forceinline__ int octet_col(int q) {
  return (q >= 4 ? RC / 2 : 0) + (((q >> 1) & 1) ? RC / 4 : 0) + ((q & 1) ? RC / 8 : 0);
}

template <int K, int CTRL, typename T>
__device__ __forceinline__ void rs_stage(T (&v)[2 * K], T (&o)[K], bool hi) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const T keep = hi ? v[K + i] : v[i];
    const T send = hi ? v[i] : v[K + i];
    o[i] = keep + dpp_mov<CTRL>(send);
  }
}

template <typename T, int RC>
__device__ __forceinline__ T octet_reduce_scatter(T (&v)[RC], int q) {
  static_assert(RC == 1 || RC == 2 || RC == 4 || RC == 8, "columns per octet");
  if constexpr (RC == 1) {
    return octet_sum(v[0]);
  } else if constexpr (RC == 2) {
    T a[1];
    rs_stage<1, 0x141>(v, a, q >= 4);
    T x = a[0];
    x += dpp_mov<0x4E>(x);
    x += dpp_mov<0xB1>(x);
    return x;
  } else if constexpr (RC == 4) {
    T a[2], b[1];
    rs_stage<2, 0x141>(v, a, q >= 4);
    rs_stage<1, 0x4E>(a, b, ((q >> 1) & 1) != 0);
    T x = b[0];
    x += dpp_mov<0xB1>(x);
    return x;
  } else {
    T a[4], b[2], c[1];
    rs_stage<4, 0x141>(v, a, q >= 4);
    rs_stage<2, 0x4E>(a, b, ((q >> 1) & 1) != 0);
    rs_stage<1, 0xB1>(b, c, (q & 1) != 0);
    return c[0];
  }
}

enum { CTR_COMPUTED = 0, CTR_HALO = 1, CTR_ERR = 3, CTR_WAVE0 = 4 };  // CTR_WAVE0 + w: compute wave w

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

// {right-hand side, dot-vector entry} pair of one column
template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  using type = double2;
};
template <>
struct Pair2<float> {
  using type = float2;
};

// Halo wavefront: entries are staged in order; lane j of a round watches entry pos + j.
// An entry is ready when its R values are no longer the sentinel and the compute wave has
// finished the steps that still read the slot's previous occupant.
// Steps computed by every compute wave: the counter CTR_COMPUTED (one compute wave, NW = 0)
// or the least of the NW per-wave counters from CTR_WAVE0 on.
template <int NW>
__device__ __forceinline__ int computed_steps(int* ctr) {
  if constexpr (NW == 0) {
    return lds_load(&ctr[CTR_COMPUTED]);
  } else {
    int m = lds_load(&ctr[CTR_WAVE0]);
#pragma unroll
    for (int w = 1; w < NW; ++w) m = min(m, lds_load(&ctr[CTR_WAVE0 + w]));
    return m;
  }
}

// LDS slot addresses of an R-column batch.  With power-of-two slot sizes every lane of a
// column block would read the same few LDS banks (the slot's low bits select nothing), so
// a 16-byte pad follows every 2^ps slots: ps = 0 (every slot; the default) or kCompact
// (every 256 / (R sizeof(T)) slots, about 6 % more LDS instead of 12-25 %, so that two
// workgroups fit one CU).  Either way the gathers of up to 16 different slots spread over
// all banks.
template <typename T, int R>
struct SlotLayout {
  static constexpr uint32_t kRow = (uint32_t)(R * sizeof(T));
  static constexpr int kCompact = R == 1 ? 0 : __builtin_ctz(256u / kRow);
  __host__ __device__ static constexpr uint32_t addr(uint32_t slot, int ps) {
    return R == 1 ? slot * kRow : slot * kRow + (slot >> ps) * 16u;
  }
  __host__ __device__ static constexpr size_t bytes(int nslots, int ps) {
    return (size_t)addr((uint32_t)nslots + 1u, ps) + 16u;
  }
};

// Rows nrows .. nrows + ncpl - 1 are coupling rows, read from cpl (R = 1 layouts only).
template <typename T, int R, int NW = 0>
__device__ __forceinline__ void halo_wave(const int32_t* __restrict__ grp_halo_ptr, const int32_t* __restrict__ halo_row,
                                          const int32_t* __restrict__ halo_slot,
                                          const int32_t* __restrict__ halo_free, int nrows, int nslots, int ld,
                                          int* err, int g, int lane, int* ctr, T* xs, const T* out,
                                          const T* cpl = nullptr, int ncpl = 0, int pad_shift = 0) {
  const int h0 = grp_halo_ptr[g], h1 = grp_halo_ptr[g + 1];
  const int nhalo = h1 - h0;
  int pos = 0;
  long spins = 0;
  while (pos < nhalo) {
    const int idx = pos + lane;
    const bool valid = idx < nhalo;
    int row = -1, slot = 0, fr = 0;
    if (valid) {
      row = halo_row[h0 + idx];
      slot = halo_slot[h0 + idx];
      fr = halo_free[h0 + idx];
    }
    const bool inb = valid && row >= 0 && row < nrows + ncpl && slot > 0 && slot < nslots;
    T v[R];
    bool ready = true;
    const T* src = nullptr;
    if (inb) {
      src = row < nrows ? out + (size_t)row * ld : cpl + (size_t)(row - nrows) * ld;
      // R > 1: one column probes the entry; the whole row is read only for the ready prefix
      // (a poll of entries that are not ready yet then costs one load per lane, not R)
      v[0] = dev_load(src);
      ready = !is_sentinel(v[0]) && computed_steps<NW>(ctr) >= fr;
    }
    unsigned long long notready = __ballot(!ready);
    int count = notready ? __ffsll((long long)notready) - 1 : 64;
    count = min(count, nhalo - pos);
    if constexpr (R > 1) {
      if (count > 0) {
        bool full = true;
        if (lane < count && inb) {
#pragma unroll
          for (int c = 1; c < R; ++c) {
            v[c] = dev_load(src + c);
            full = full && !is_sentinel(v[c]);
          }
        }
        notready = __ballot(!full);
        if (notready) count = min(count, __ffsll((long long)notready) - 1);
      }
    }
    if (count == 0) {
      ++spins;
      if ((spins & 63) == 0 && (spins > (kSpinLimit >> 6) || err_set(err) || lds_load(&ctr[CTR_ERR]) != 0)) {
        if (spins > (kSpinLimit >> 6)) raise_err(err);
        if (lane == 0) {
          lds_signal(&ctr[CTR_ERR], 1);
          lds_signal(&ctr[CTR_HALO], nhalo);
        }
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    if (lane < count && inb) {
      T* xp = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(xs) + SlotLayout<T, R>::addr((uint32_t)slot, pad_shift));
#pragma unroll
      for (int c = 0; c < R; ++c) xp[c] = v[c];
    }
    pos += count;
    if (lane == 0) lds_signal(&ctr[CTR_HALO], pos);
  }
}

// The last group's sum of the group partials partials[k R + c] (k < ngroups, c < R), by the
// 64 lanes of one wavefront: lane l takes column l % R and groups l / R, l / R + 64 / R, ...,
// then a fixed shuffle tree joins the lanes of a column (the same order on every run); lane
// c < R writes out[c].  The lanes' loads are independent, so the tail is a few memory
// latencies instead of one per group.
template <int R>
__device__ __forceinline__ void last_group_sum(const double* partials, int ngroups, double* out, int lane) {
  static_assert(R >= 1 && 64 % R == 0, "R divides the wavefront");
  constexpr int P = 64 / R;  // lanes per column
  const int c = lane % R, j = lane / R;
  double v = 0.0;
#pragma unroll 4
  for (int k = j; k < ngroups; k += P) v += dev_load(partials + (size_t)k * R + c);
#pragma unroll
  for (int off = 32; off >= R; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane < R) out[lane] = v;
}

// Prefetch depth (steps in flight) of the single-wave batched kernel: for R = 1 as deep as the
// 63 outstanding vector memory operations (about 7 to 10 per step) and the register file
// allow; with R columns the per-step records are R times larger and the depth is small.
constexpr int batch_depth(int R, int EP, int tsize) {
  return EP <= 4 ? (R == 1 ? 9 : (R == 8 ? 3 : 2))
       : EP <= 8 ? (R == 1 ? (tsize == 8 ? 7 : 8) : (R == 8 ? 3 : 2))
       : EP <= 12 ? (R == 1 ? 4 : 2)
                  : (R == 1 ? 3 : 2);
}

// Prefetch depth of the column-split kernel (GC 16-byte gathers per entry and wave).
constexpr int cols_depth(int GC, int EP) {
  return GC == 1 ? (EP <= 4 ? 7 : (EP <= 8 ? 5 : (EP <= 12 ? 3 : 2))) : (EP <= 4 ? 5 : (EP <= 8 ? 3 : 2));
}

template <typename T, int R, int EP, int D>
__global__ __launch_bounds__(kTrsvThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trsv(
    TrsvArgs a, const T* __restrict__ sval, const typename RowRec<T>::type* __restrict__ srinfo,
    const T* __restrict__ rd_s, T* __restrict__ out, T* __restrict__ dummy, int with_dot,
    double* __restrict__ dot_out, const int* __restrict__ skip) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int NV = EP / VN;  // vector loads of factor values per lane and step
  using SL = SlotLayout<T, R>;  // slot id -> byte offset in xs
  extern __shared__ __align__(16) unsigned char smem[];
  if (skip != nullptr && *skip) return;
  int* ctr = reinterpret_cast<int*>(smem);
  T* xs = reinterpret_cast<T*>(smem + 64);

  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  const int s0 = a.grp_step_ptr[g], s1 = a.grp_step_ptr[g + 1];
  const int nsteps = s1 - s0;
  if (tid < 16) ctr[tid] = 0;
  if (tid < R) xs[tid] = T(0);  // slot 0: the zero slot read by padding entries
  __syncthreads();

  double dotacc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) dotacc[c] = 0.0;

  if (wid == 0) {
    // ------------------------------ compute wave ------------------------------
    // the group's entries per lane: 4, or the schedule's widest (EP)
    auto compute = [&](auto ep_c) {
    constexpr int EPX = decltype(ep_c)::value;
    constexpr int NVX = EPX / VN;
    constexpr int DX = EPX == EP ? D : batch_depth(R, EPX, sizeof(T));
    const int q = lane % kTrsvG;
    // padding rows and steps past the end store to a word of the workgroup's own (64 words
    // per workgroup, kTrsvDummyGroups blocks; the lanes of a wavefront share theirs):
    // device-scope stores of many workgroups to one shared word serialise
    T* const dummy_l = dummy + (size_t)(g % kTrsvDummyGroups) * 64;
    const int r = lane / kTrsvG;
    V pv[DX][NVX];
    uint4 ps[DX][EPX / 4];
    typename RowRec<T>::type pri[DX];
    T prd[DX][2 * R];  // {right-hand side, dot-vector entry} of each column
    int prow[DX];
    int halo_seen = 0;
    // per-lane parts of the record addresses; the step part stays scalar
    const int64_t eoff = a.grp_eoff[g] - (int64_t)s0 * 64 * EPX;  // step ss at eoff + ss * 64 * EPX
    const T* sval_l = sval + eoff + (size_t)lane * EPX;
    const uint32_t* ssrc_l = a.ssrc + eoff + (size_t)lane * EPX;
    const typename RowRec<T>::type* sri_l = srinfo + r;
    const T* rd_l = rd_s + (size_t)r * 2 * R;
    const int32_t* srow_l = a.srow + r;
    auto load = [&](int d, int ss) {
      const V* vp = reinterpret_cast<const V*>(sval_l + (size_t)ss * 64 * EPX);
#pragma unroll
      for (int k = 0; k < NVX; ++k) pv[d][k] = vp[k];
      const uint4* sp = reinterpret_cast<const uint4*>(ssrc_l + (size_t)ss * 64 * EPX);
#pragma unroll
      for (int k = 0; k < EPX / 4; ++k) ps[d][k] = sp[k];
      pri[d] = sri_l[(size_t)ss * kTrsvRPS];
#pragma unroll
      for (int c = 0; c < 2 * R; ++c) prd[d][c] = rd_l[(size_t)ss * kTrsvRPS * 2 * R + c];
      prow[d] = srow_l[(size_t)ss * kTrsvRPS];
    };
    // Software pipeline over D register buffers: during step ss (buffer d) the wave
    // issues the step's LDS gathers, then the loads of step ss + D - 1 into the buffer
    // the previous step used, then waits for the gathers (R = 1; with R columns the
    // loads follow the accumulation).  The global memory operations are issued on every
    // path and in buffer order (step index clamped to the last step; scheduling barriers
    // keep each buffer's loads together, in the prologue as in the loop), and the loop
    // sits inside the prologue's branch as a do-while: the number of operations in
    // flight after each buffer's loads is then the same on every path into a use, so the
    // compiler's vmcnt waits hold back only the buffer about to be used.  Steps past the
    // end of the group (last round) recompute the last step on its clamped records and
    // store to a dummy location.
    if (nsteps > 0) {
#pragma unroll
      for (int d = 0; d + 1 < DX; ++d) {
        load(d, min(s0 + d, s1 - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
      int s = s0;
      do {
#pragma unroll
        for (int d = 0; d < DX; ++d) {
          const int ss = s + d;
          const int k = ss - s0;
          const bool live = ss < s1;
          if (live && pri[d].need > halo_seen)
            halo_seen = lds_wait<false, false>(&ctr[CTR_HALO], pri[d].need, &ctr[CTR_ERR], a.err);
          // two interleaved FMA chains (even / odd entries) halve the dependency latency
          T acc[R], acc2[R];
#pragma unroll
          for (int c = 0; c < R; ++c) acc[c] = acc2[c] = T(0);
          auto xaddr = [&](int e) {
            const unsigned src = reinterpret_cast<const unsigned*>(&ps[d][e / 4])[e % 4];
            return reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(xs) + SL::addr(src, 0));
          };
          if constexpr (R == 1) {
            // gathers first, the next loads while they are in flight, then the FMAs
            T xv[EPX];
#pragma unroll
            for (int e = 0; e < EPX; ++e) xv[e] = *xaddr(e);
            __builtin_amdgcn_sched_barrier(0);
            load((d + DX - 1) % DX, min(ss + DX - 1, s1 - 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = 0; e < EPX; ++e) {
              const T v = reinterpret_cast<const T*>(&pv[d][e / VN])[e % VN];
              if (e & 1)
                acc2[0] = fma(v, xv[e], acc2[0]);
              else
                acc[0] = fma(v, xv[e], acc[0]);
            }
          } else {
            // R columns per entry: gather and accumulate entry by entry (register budget)
#pragma unroll
            for (int e = 0; e < EPX; ++e) {
              const T v = reinterpret_cast<const T*>(&pv[d][e / VN])[e % VN];
              const T* xp = xaddr(e);
              if (e & 1) {
#pragma unroll
                for (int c = 0; c < R; ++c) acc2[c] = fma(v, xp[c], acc2[c]);
              } else {
#pragma unroll
                for (int c = 0; c < R; ++c) acc[c] = fma(v, xp[c], acc[c]);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
            load((d + DX - 1) % DX, min(ss + DX - 1, s1 - 1));
            __builtin_amdgcn_sched_barrier(0);
          }
          // Every lane of the octet holds the row's sum and result.  Rows whose value no
          // later step reads carry the dummy slot (nslots), so the slot store needs no
          // branch; the global store is issued on every path (padding rows and steps past
          // the end write to the dummy location).
          T res[R];
#pragma unroll
          for (int c = 0; c < R; ++c) res[c] = (prd[d][2 * c] - octet_sum(acc[c] + acc2[c])) * pri[d].dinv;
          const bool real = live && prow[d] >= 0;
          T* gp = !real ? dummy_l
                  : prow[d] < a.nrows ? out + (size_t)prow[d] * a.ld
                                      : reinterpret_cast<T*>(a.cpl) + (size_t)(prow[d] - a.nrows) * a.ld;
          if constexpr (R == 1) {
            dev_store(gp, res[0]);
          } else {
            // lane q of the octet stores columns q, q + 8, ... (R is a multiple of 8)
#pragma unroll
            for (int c = 0; c < R; c += kTrsvG) {
              T v = res[c];
#pragma unroll
              for (int j = 1; j < kTrsvG; ++j)
                if (q == j) v = res[c + j];
              dev_store(gp + (real ? c + q : 0), v);
            }
          }
          if (live) {
            if (q == 0 && prow[d] >= 0) {
#pragma unroll
              for (int c = 0; c < R; ++c) dotacc[c] += (double)res[c] * (double)prd[d][2 * c + 1];
            }
            T* xp = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(xs) + SL::addr((uint32_t)pri[d].slot, 0));
            if constexpr (R == 1) {
              xp[0] = res[0];
              lds_signal(&ctr[CTR_COMPUTED], k + 1);
            } else {
              if (q == 0) {
#pragma unroll
                for (int c = 0; c < R; ++c) xp[c] = res[c];
              }
              if (lane == 0) lds_signal(&ctr[CTR_COMPUTED], k + 1);
            }
          }
        }
        s += DX;
      } while (s < s1);
    }
    };
    if (a.grp_ep[g] == EP)
      compute(std::integral_constant<int, EP>{});
    else
      compute(std::integral_constant<int, 4>{});
  } else {
    // ------------------------------- halo wave --------------------------------
    halo_wave<T, R>(a.grp_halo_ptr, a.halo_row, a.halo_slot, a.halo_free, a.nrows, a.nslots, a.ld, a.err, g, lane,
                    ctr, xs, out, reinterpret_cast<const T*>(a.cpl), a.ncpl, 0);
  }
  __syncthreads();
  if (tid == 0 && lds_load(&ctr[CTR_ERR]) != 0) raise_err(a.err);

  // ------------------------- epilogue: fused dot product -------------------------
  // The compute wave stores the group's dot partials (device scope), waits for their
  // acknowledgement and takes a ticket; the last group adds the partials (last_group_sum).
  if (with_dot && wid == 0) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double v = dotacc[c];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) dev_store(a.partials + (size_t)g * R + c, v);
    }
    unsigned int prev = 0;
    if (lane == 0) {
      wait_vm_stores();
      prev = __hip_atomic_fetch_add(a.done_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = (unsigned int)__shfl((int)prev, 0, 64);
    if (prev == (unsigned int)(a.ngroups - 1)) {
      last_group_sum<R>(a.partials, a.ngroups, dot_out, lane);
      if (lane == 0) __hip_atomic_store(a.done_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Batched solve with the columns split over W compute wavefronts plus the halo wavefront.
// Compute wave w owns columns [w RC, (w + 1) RC), RC = R / W, so each dependency is G =
// RC / (16 bytes of T) 16-byte LDS gathers and a step issues all its gathers before the
// FMAs, as the single-column step does.  The waves walk the same steps and read the same
// factor records; they share no values (each reads and writes only its own columns of the
// LDS slots), so they run independently.  The halo wave refills a slot only after every
// compute wave has finished the steps that read its previous occupant (least of the
// per-wave counters).
// ---------------------------------------------------------------------------
template <typename T, int R, int EP, int D, int W, int PS>
__global__ __launch_bounds__(64 * (W + 1)) void k_trsv_cols(
    TrsvArgs a, const T* __restrict__ sval, const typename RowRec<T>::type* __restrict__ srinfo,
    const T* __restrict__ rd_s, T* __restrict__ out, T* __restrict__ dummy, int with_dot,
    double* __restrict__ dot_out, const int* __restrict__ skip) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  constexpr int RC = R / W;
  constexpr int G = RC / VN;  // 16-byte gathers per entry
  static_assert(G >= 1 && G * VN == RC && W * RC == R && W <= 8 && D >= 2, "column split");
  constexpr int NV = EP / VN;
  using SL = SlotLayout<T, R>;  // slot id -> byte offset in xs
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sdot[R];
  if (skip != nullptr && *skip) return;
  int* ctr = reinterpret_cast<int*>(smem);
  T* xs = reinterpret_cast<T*>(smem + 64);

  // The launch may hold several column blocks of R columns each (a wide batch solved as
  // independent R-column solves side by side): block b is group b % ngroups of column
  // block b / ngroups, with its own columns, gathered pairs, dot partials and ticket.
  const int g = blockIdx.x % a.ngroups;
  const int hc = blockIdx.x / a.ngroups;
  out += (size_t)hc * R;
  rd_s += (size_t)hc * a.nrow_slots * 2 * R;
  T* const cplh = reinterpret_cast<T*>(a.cpl) + (size_t)hc * R;
  double* const partials_h = a.partials + (size_t)hc * a.ngroups * R;
  unsigned int* const done_h = a.done_count + hc;
  if (dot_out != nullptr) dot_out += hc * R;
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  const int s0 = a.grp_step_ptr[g], s1 = a.grp_step_ptr[g + 1];
  if (tid < 16) ctr[tid] = 0;
  if (tid < R) {
    xs[tid] = T(0);  // slot 0: the zero slot read by padding entries
    sdot[tid] = 0.0;
  }
  __syncthreads();

  if (wid < W) {
    // ------------------------------ compute waves -----------------------------
    const int cb = wid * RC;
    const int q = lane % kTrsvG;
    // padding rows and steps past the end store to a word of the workgroup's own (64 words
    // per workgroup, kTrsvDummyGroups blocks; the lanes of a wavefront share theirs):
    // device-scope stores of many workgroups to one shared word serialise
    T* const dummy_l = dummy + (size_t)(blockIdx.x % kTrsvDummyGroups) * 64;
    const int r = lane / kTrsvG;
    // the octet's reduce-scatter leaves column cq of the row in this lane; the first of the
    // 8 / RC lanes with that column (lead) writes its LDS slot entry and accumulates its dot
    const int cq = octet_col<RC>(q);
    const bool lead = (q & (kTrsvG / RC - 1)) == 0;
    double dotacc = 0.0;
    // the group's entries per lane: 4, or the schedule's widest (EP)
    auto compute = [&](auto ep_c) {
    constexpr int EPX = decltype(ep_c)::value;
    constexpr int NVX = EPX / VN;
    constexpr int DX = EPX == EP ? D : cols_depth(G, EPX);
    using P = typename Pair2<T>::type;
    V pv[DX][NVX];
    uint4 ps[DX][EPX / 4];
    typename RowRec<T>::type pri[DX];
    P prd[DX];  // {right-hand side, dot-vector entry} of this lane's column
    int prow[DX];
    int halo_seen = 0;
    const int64_t eoff = a.grp_eoff[g] - (int64_t)s0 * 64 * EPX;  // step ss at eoff + ss * 64 * EPX
    const T* sval_l = sval + eoff + (size_t)lane * EPX;
    const uint32_t* ssrc_l = a.ssrc + eoff + (size_t)lane * EPX;
    const typename RowRec<T>::type* sri_l = srinfo + r;
    const T* rd_l = rd_s + ((size_t)r * R + cb + cq) * 2;
    const int32_t* srow_l = a.srow + r;
    auto load = [&](int d, int ss) {
      const V* vp = reinterpret_cast<const V*>(sval_l + (size_t)ss * 64 * EPX);
#pragma unroll
      for (int k = 0; k < NVX; ++k) pv[d][k] = vp[k];
      const uint4* sp = reinterpret_cast<const uint4*>(ssrc_l + (size_t)ss * 64 * EPX);
#pragma unroll
      for (int k = 0; k < EPX / 4; ++k) ps[d][k] = sp[k];
      pri[d] = sri_l[(size_t)ss * kTrsvRPS];
      prd[d] = *reinterpret_cast<const P*>(rd_l + (size_t)ss * kTrsvRPS * 2 * R);
      prow[d] = srow_l[(size_t)ss * kTrsvRPS];
    };
    // The same software pipeline as the single-wave kernel: D register buffers, the loads
    // of step ss + D - 1 issued between the gathers of step ss and their use.
    if (s1 > s0) {
#pragma unroll
      for (int d = 0; d + 1 < DX; ++d) {
        load(d, min(s0 + d, s1 - 1));
        __builtin_amdgcn_sched_barrier(0);
      }
      int s = s0;
      do {
#pragma unroll
        for (int d = 0; d < DX; ++d) {
          const int ss = s + d;
          const int k = ss - s0;
          const bool live = ss < s1;
          if (live && pri[d].need > halo_seen)
            halo_seen = lds_wait<false, false>(&ctr[CTR_HALO], pri[d].need, &ctr[CTR_ERR], a.err);
          V xv[EPX][G];
#pragma unroll
          for (int e = 0; e < EPX; ++e) {
            const unsigned src = reinterpret_cast<const unsigned*>(&ps[d][e / 4])[e % 4];
            const V* xp = reinterpret_cast<const V*>(reinterpret_cast<const unsigned char*>(xs + cb) + SL::addr(src, PS));
#pragma unroll
            for (int k = 0; k < G; ++k) xv[e][k] = xp[k];
          }
          __builtin_amdgcn_sched_barrier(0);
          load((d + DX - 1) % DX, min(ss + DX - 1, s1 - 1));
          __builtin_amdgcn_sched_barrier(0);
          T acc[RC], acc2[RC];
#pragma unroll
          for (int c = 0; c < RC; ++c) acc[c] = acc2[c] = T(0);
#pragma unroll
          for (int e = 0; e < EPX; ++e) {
            const T v = reinterpret_cast<const T*>(&pv[d][e / VN])[e % VN];
            const T* xe = reinterpret_cast<const T*>(&xv[e][0]);
#pragma unroll
            for (int c = 0; c < RC; ++c) {
              if (e & 1)
                acc2[c] = fma(v, xe[c], acc2[c]);
              else
                acc[c] = fma(v, xe[c], acc[c]);
            }
          }
          T part[RC];
#pragma unroll
          for (int c = 0; c < RC; ++c) part[c] = acc[c] + acc2[c];
          const T res = (prd[d].x - octet_reduce_scatter<T, RC>(part, q)) * pri[d].dinv;
          // every lane stores its column (lanes with the same column store the same value;
          // padding rows and steps past the end store to the dummy location), so the store
          // is issued on every path
          static_assert(RC <= kTrsvG, "one column per lane of the octet");
          const bool real = live && prow[d] >= 0;
          T* gp = !real ? dummy_l + cb
                  : prow[d] < a.nrows ? out + (size_t)prow[d] * a.ld + cb + cq
                                      : cplh + (size_t)(prow[d] - a.nrows) * a.ld + cb + cq;
          dev_store(gp, res);
          if (live) {
            if (lead) {
              if (prow[d] >= 0) dotacc += (double)res * (double)prd[d].y;
              T* xp = reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(xs) + SL::addr((uint32_t)pri[d].slot, PS)) + cb;
              xp[cq] = res;
            }
            if (lane == 0) lds_signal(&ctr[CTR_WAVE0 + wid], k + 1);
          }
        }
        s += DX;
      } while (s < s1);
    }
    };
    if (a.grp_ep[g] == EP)
      compute(std::integral_constant<int, EP>{});
    else
      compute(std::integral_constant<int, 4>{});
    if (with_dot) {
#pragma unroll
      for (int c = 0; c < RC; ++c) {
        double v = (lead && cq == c) ? dotacc : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sdot[cb + c] = v;
      }
    }
  } else {
    // ------------------------------- halo wave --------------------------------
    halo_wave<T, R, W>(a.grp_halo_ptr, a.halo_row, a.halo_slot, a.halo_free, a.nrows, a.nslots, a.ld, a.err, g,
                       lane, ctr, xs, out, cplh, a.ncpl, PS);
  }
  __syncthreads();
  if (tid == 0 && lds_load(&ctr[CTR_ERR]) != 0) raise_err(a.err);

  // fused dot product: the group's partials of all R columns (device scope), then a ticket;
  // the last group adds the partials (last_group_sum)
  if (with_dot && wid == 0) {
    if (lane < R) dev_store(partials_h + (size_t)g * R + lane, sdot[lane]);
    unsigned int prev = 0;
    if (lane == 0) {
      wait_vm_stores();
      prev = __hip_atomic_fetch_add(done_h, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = (unsigned int)__shfl((int)prev, 0, 64);
    if (prev == (unsigned int)(a.ngroups - 1)) {
      last_group_sum<R>(partials_h, a.ngroups, dot_out, lane);
      if (lane == 0) __hip_atomic_store(done_h, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Single-column solve on the per-group block layout (one right-hand side, contiguous
// vectors).  Same protocol as k_trsv with R = 1; the compute wave's step is trimmed to
// what the arithmetic needs: every record of a step is read relative to one scalar block
// address (row records, step header, LDS byte addresses and factor values) plus the
// per-solve {rhs, dot} pair, the gathers use the stored LDS byte addresses as they are,
// padding rows and tail steps repeat real ones (no per-step branches), and a single wait
// covers the step's gathers.
// ---------------------------------------------------------------------------
struct FastArgs {
  const int32_t* grp_step_ptr;
  const int32_t* grp_npad;
  const int32_t* grp_ep;
  const int64_t* grp_blk;
  const unsigned char* blk;
  const int32_t* grp_halo_ptr;
  const int32_t* halo_row;
  const int32_t* halo_slot;
  const int32_t* halo_free;
  const int32_t* grp_cpl;
  void* cpl;
  unsigned int* done_count;
  int* err;
  double* partials;
  int ngroups;
  int nslots;
  int nrows;
  int ncpl;
};

template <typename T>
struct FastDyn {
  T rhs, dot;
};
template <typename T>
struct FastRec;
template <>
struct FastRec<double> {
  using type = FastRec64;
  static __device__ __forceinline__ uint32_t slot(const FastRec64& r) { return r.slot_need & 0xffffu; }
  static __device__ __forceinline__ int need(const FastRec64& r) { return (int)(r.slot_need >> 16); }
};
template <>
struct FastRec<float> {
  using type = FastRec32;
  static __device__ __forceinline__ uint32_t slot(const FastRec32& r) { return (uint32_t)r.slot_byte; }
  static __device__ __forceinline__ int need(const FastRec32& r) { return r.need; }
};

// Buffer resources (raw, byte-addressed, bounds-checked against num_records) let every load
// of a step take its per-step part from one scalar offset and its per-lane part from a
// register computed once.
constexpr int kBufferFlags = 0x00020000;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kStoreSc1 = 16;  // cache policy of device-scope stores (visible across the XCDs)
constexpr int kWaitLgkm0 = 0xC07F;  // s_waitcnt lgkmcnt(0), no vmcnt / expcnt wait (gfx9 encoding)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kBufferFlags);
}

// LDS access by byte address: dynamic shared memory starts at LDS address 0 in these
// kernels (they declare no static shared memory; checked at kernel entry).
template <typename T>
__device__ __forceinline__ T lds_at(uint32_t addr) {
  return *reinterpret_cast<const __attribute__((address_space(3))) T*>((size_t)addr);
}
template <typename T>
__device__ __forceinline__ void lds_put(uint32_t addr, T v) {
  *reinterpret_cast<__attribute__((address_space(3))) T*>((size_t)addr) = v;
}

// Group metadata loaded through vector loads is not known to be uniform: move it to
// scalar registers (the buffer resources built from it must live there).
__device__ __forceinline__ int uniform32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T from_bits2(u32x2 b) {
  return __builtin_bit_cast(T, b);
}

template <typename T, int EP, int D, bool kDot>
__device__ __forceinline__ double fast_compute(const FastArgs& a, const FastDyn<T>* __restrict__ dyn,
                                               T* __restrict__ out, unsigned char* smem, int g, int lane) {
  using Rec = typename FastRec<T>::type;
  constexpr int SB = fast_block_bytes<T>(EP);
  constexpr int OFF_SLOT = kFastHdr;
  constexpr int OFF_VAL = kFastHdr + 64 * EP * 4;
  constexpr int NVL = EP * (int)sizeof(T) / 16;  // 16-byte loads of values per lane and step
  constexpr int DYN = kTrsvRPS * (int)sizeof(FastDyn<T>);
  int* ctr = reinterpret_cast<int*>(smem);
  const int s0 = uniform32(a.grp_step_ptr[g]);
  const int nalloc = uniform32(a.grp_step_ptr[g + 1]) - s0;
  const int npad = uniform32(a.grp_npad[g]);
  const int64_t b0 = uniform64(a.grp_blk[g]), b1 = uniform64(a.grp_blk[g + 1]);
  const __amdgpu_buffer_rsrc_t rb = make_rsrc(a.blk + b0, (uint32_t)(b1 - b0));
  const __amdgpu_buffer_rsrc_t rd = make_rsrc(dyn + (size_t)s0 * kTrsvRPS, (uint32_t)nalloc * DYN);
  // a group's rows are all rows of the factor or all coupling rows (stored apart)
  const bool cgrp = uniform32(a.grp_cpl[g]) != 0;
  const __amdgpu_buffer_rsrc_t ro = cgrp ? make_rsrc(a.cpl, (uint32_t)a.ncpl * (uint32_t)sizeof(T))
                                         : make_rsrc(out, (uint32_t)a.nrows * (uint32_t)sizeof(T));
  const int r = lane / kTrsvG;
  const uint32_t o_rec = (uint32_t)r * 16u;
  const uint32_t o_slot = (uint32_t)(OFF_SLOT + lane * EP * 4);
  const uint32_t o_val = (uint32_t)(OFF_VAL + lane * EP * (int)sizeof(T));
  const uint32_t o_dyn = (uint32_t)r * (uint32_t)sizeof(FastDyn<T>);
  u32x4 pv[D][NVL];
  u32x4 ps[D][EP / 4];
  u32x4 prc[D];
  FastDyn<T> pdy[D];
  auto load = [&](int d, int j) {
    const int sb = j * SB, sd = j * DYN;
#pragma unroll
    for (int k = 0; k < NVL; ++k) pv[d][k] = __builtin_amdgcn_raw_buffer_load_b128(rb, o_val + 16 * k, sb, 0);
#pragma unroll
    for (int k = 0; k < EP / 4; ++k) ps[d][k] = __builtin_amdgcn_raw_buffer_load_b128(rb, o_slot + 16 * k, sb, 0);
    prc[d] = __builtin_amdgcn_raw_buffer_load_b128(rb, o_rec, sb, 0);
    if constexpr (sizeof(T) == 8) {
      const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(rd, o_dyn, sd, 0);
      pdy[d].rhs = from_bits2<T>(t.xy);
      pdy[d].dot = from_bits2<T>(t.zw);
    } else {
      const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(rd, o_dyn, sd, 0);
      const unsigned w0 = t.x, w1 = t.y;  // components copied out first (see below)
      pdy[d].rhs = __builtin_bit_cast(T, w0);
      pdy[d].dot = __builtin_bit_cast(T, w1);
    }
  };
  double dacc = 0.0;
  int halo_seen = 0;
  if (npad > 0) {
#pragma unroll
    for (int d = 0; d + 1 < D; ++d) {
      load(d, d);
      __builtin_amdgcn_sched_barrier(0);
    }
    int j = 0;
    do {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int jj = j + d;
        const Rec rec = __builtin_bit_cast(Rec, prc[d]);
        const int need = __builtin_amdgcn_readfirstlane(FastRec<T>::need(rec));
        if (need > halo_seen)
          halo_seen = __builtin_amdgcn_readfirstlane(
              lds_wait<false, false>(&ctr[CTR_HALO], need, &ctr[CTR_ERR], a.err));
        T xv[EP];
#pragma unroll
        for (int e = 0; e < EP; ++e) xv[e] = lds_at<T>(ps[d][e / 4][e % 4]);
        __builtin_amdgcn_sched_barrier(0);
        load((d + D - 1) % D, jj + D - 1);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);  // one wait for all gathers
        __builtin_amdgcn_sched_barrier(0);
        T acc = T(0), acc2 = T(0);
#pragma unroll
        for (int e = 0; e < EP; ++e) {
          T v;
          if constexpr (sizeof(T) == 8) {
            const u32x4 w = pv[d][e / 2];
            v = from_bits2<T>((e & 1) ? w.zw : w.xy);
          } else {
            // copy the component out first: clang's bit cast of a vector component
            // expression reads component 0 whatever the index
            const unsigned w = pv[d][e / 4][e % 4];
            v = __builtin_bit_cast(T, w);
          }
          if (e & 1)
            acc2 = fma(v, xv[e], acc2);
          else
            acc = fma(v, xv[e], acc);
        }
        const T res = (pdy[d].rhs - octet_sum(acc + acc2)) * rec.dinv;
        if constexpr (sizeof(T) == 8)
          __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, res), ro, (uint32_t)rec.row_byte, 0,
                                                kStoreSc1);
        else
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, res), ro, (uint32_t)rec.row_byte, 0,
                                                kStoreSc1);
        if (kDot) dacc = fma((double)res, (double)pdy[d].dot, dacc);
        lds_put<T>(FastRec<T>::slot(rec), res);
        lds_signal(&ctr[CTR_COMPUTED], jj + 1);
      }
      j += D;
    } while (j < npad);
  }
  return dacc;
}

template <typename T, bool kDot>
__global__ __launch_bounds__(kTrsvThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_trsv_fast(
    FastArgs a, const FastDyn<T>* __restrict__ dyn, T* __restrict__ out, double* __restrict__ dot_out,
    const int* __restrict__ skip) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (skip != nullptr && *skip) return;
  int* ctr = reinterpret_cast<int*>(smem);
  T* xs = reinterpret_cast<T*>(smem + 64);
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  if ((uint32_t)(size_t)(__attribute__((address_space(3))) void*)smem != 0u) {  // see lds_at
    if (tid == 0) raise_err(a.err);
    return;
  }
  if (tid < 16) ctr[tid] = 0;
  if (tid == 0) xs[0] = T(0);  // slot 0: the zero slot read by padding entries
  __syncthreads();
  double dacc = 0.0;
  if (wid == 0) {
    if (uniform32(a.grp_ep[g]) == 4)
      dacc = fast_compute<T, 4, fast_depth(4), kDot>(a, dyn, out, smem, g, lane);
    else
      dacc = fast_compute<T, 8, fast_depth(8), kDot>(a, dyn, out, smem, g, lane);
  } else {
    halo_wave<T, 1>(a.grp_halo_ptr, a.halo_row, a.halo_slot, a.halo_free, a.nrows, a.nslots, 1, a.err, g, lane, ctr,
                    xs, out, reinterpret_cast<const T*>(a.cpl), a.ncpl);
  }
  __syncthreads();
  if (tid == 0 && lds_load(&ctr[CTR_ERR]) != 0) raise_err(a.err);
  if (kDot && wid == 0) {
    // every lane of an octet accumulated its row: the wave sum counts each row 8 times
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) dacc += __shfl_xor(dacc, off, 64);
    dacc *= 1.0 / kTrsvG;
    unsigned int prev = 0;
    if (lane == 0) {
      dev_store(a.partials + g, dacc);
      wait_vm_stores();
      prev = __hip_atomic_fetch_add(a.done_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = (unsigned int)__shfl((int)prev, 0, 64);
    if (prev == (unsigned int)(a.ngroups - 1)) {
      last_group_sum<1>(a.partials, a.ngroups, dot_out, lane);
      if (lane == 0) __hip_atomic_store(a.done_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Per-solve {rhs, dot} pairs in the single-column step order (repeats carry dot = 0) and
// the output rows reset to the sentinel.  Coupling rows (row >= nrows) have right-hand side
// and dot entry 0; their outputs in cpl are reset too.
template <typename T>
__global__ void k_fast_gather_dyn(int64_t nrow_slots, const int32_t* __restrict__ srow2, const T* __restrict__ rhs,
                                  const T* __restrict__ dotv, FastDyn<T>* __restrict__ dyn, T* __restrict__ out,
                                  T* __restrict__ cpl, int nrows, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nrow_slots;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int r2 = srow2[k];
    const int row = r2 >= 0 ? r2 : ~r2;
    FastDyn<T> v;
    if (row < nrows) {
      v.rhs = rhs[row];
      v.dot = (r2 >= 0 && dotv != nullptr) ? dotv[row] : T(0);
      if (r2 >= 0) out[row] = sentinel_value<T>();
    } else {
      v.rhs = T(0);
      v.dot = T(0);
      if (r2 >= 0) cpl[row - nrows] = sentinel_value<T>();
    }
    dyn[k] = v;
  }
}

// Factor values and reciprocal diagonals into the single-column blocks (both precisions):
// one thread per (step, lane).
__global__ void k_fast_gather_static(int64_t nsteps, const int64_t* __restrict__ step_val64,
                                     const int64_t* __restrict__ step_val32, const int32_t* __restrict__ step_ep,
                                     const int32_t* __restrict__ vperm, const int32_t* __restrict__ dsrc,
                                     const double* __restrict__ Lval, unsigned char* __restrict__ blk64,
                                     unsigned char* __restrict__ blk32) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nsteps * 64;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = t / 64;
    const int lane = int(t % 64);
    const int ep = step_ep[s];
    double* v64 = reinterpret_cast<double*>(blk64 + step_val64[s]) + lane * ep;
    float* v32 = reinterpret_cast<float*>(blk32 + step_val32[s]) + lane * ep;
    for (int e = 0; e < ep; ++e) {
      const int32_t p = vperm[(s * 64 + lane) * 8 + e];
      const double v = p >= 0 ? Lval[p] : (p == (int32_t)kTrsvValOne ? 1.0 : 0.0);
      v64[e] = v;
      v32[e] = (float)v;
    }
    if (lane < kTrsvRPS) {
      const int32_t p = dsrc[s * kTrsvRPS + lane];
      FastRec64* r64 = reinterpret_cast<FastRec64*>(blk64 + step_val64[s] - (kFastHdr + 64 * ep * 4)) + lane;
      FastRec32* r32 = reinterpret_cast<FastRec32*>(blk32 + step_val32[s] - (kFastHdr + 64 * ep * 4)) + lane;
      const double dinv = p >= 0 ? 1.0 / Lval[p] : (p == (int32_t)kTrsvValMinusOne ? -1.0 : 0.0);
      r64->dinv = dinv;
      r32->dinv = p >= 0 ? 1.0f / (float)Lval[p] : (float)dinv;
    }
  }
}

template <typename T, int R>
size_t trsv_shmem_t(int nslots, bool compact = false);

template <typename T>
static hipError_t launch_trsv_fast(const TrsvSchedDev& S, const T* rhs, T* out, const T* dotv, double* dot_out,
                                   const int* skip, hipStream_t st, const TrsvTiming* tm) {
  const TrsvFastDev& F = S.fast;
  FastArgs a;
  a.grp_step_ptr = F.grp_step_ptr;
  a.grp_npad = F.grp_npad;
  a.grp_ep = F.grp_ep;
  a.grp_blk = sizeof(T) == 8 ? F.grp_blk64 : F.grp_blk32;
  a.blk = sizeof(T) == 8 ? F.blk64 : F.blk32;
  a.grp_halo_ptr = F.grp_halo_ptr;
  a.halo_row = F.halo_row;
  a.halo_slot = F.halo_slot;
  a.halo_free = F.halo_free;
  a.grp_cpl = F.grp_cpl;
  a.cpl = F.cpl;
  a.done_count = F.done_count;
  a.err = S.err;
  a.partials = F.partials;
  a.ngroups = F.ngroups;
  a.nslots = F.nslots;
  a.nrows = F.nrows;
  a.ncpl = F.ncpl;
  FastDyn<T>* dyn = reinterpret_cast<FastDyn<T>*>(F.dyn);
  hipLaunchKernelGGL(k_fast_gather_dyn<T>, dim3(1024), dim3(256), 0, st, (int64_t)F.nsteps * kTrsvRPS, F.srow2, rhs,
                     dotv, dyn, out, reinterpret_cast<T*>(F.cpl), F.nrows, skip);
  const size_t shmem = trsv_shmem_t<T, 1>(F.nslots);
  const void* fn = dotv != nullptr ? (const void*)k_trsv_fast<T, true> : (const void*)k_trsv_fast<T, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const FastDyn<T>* dync = dyn;
  void* args[] = {&a, &dync, &out, &dot_out, &skip};
  if (tm && tm->before) (void)hipEventRecord(tm->before, st);
  e = hipLaunchKernel(fn, dim3(F.ngroups), dim3(kTrsvThreads), args, shmem, st);
  if (tm && tm->after) (void)hipEventRecord(tm->after, st);
  return e;
}

// Per-solve gather into schedule order, rd_s[((step*RPS + r)*R + c)*2] = rhs[row*ld + c] and
// rd_s[... + 1] = dotv[row*ld + c] (0 without a dot vector), and the output rows reset to
// the sentinel (R columns of a batch of width ld; the pointers carry the column offset).
template <typename T, int R>
__global__ void k_trsv_gather_rhs(int64_t nrow_slots, const int32_t* __restrict__ srow, const T* __restrict__ rhs,
                                  const T* __restrict__ dotv, int ld, T* __restrict__ rd_s, T* __restrict__ out,
                                  T* __restrict__ cpl, int nrows, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nrow_slots * R;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = t / R;
    const int c = int(t % R);
    const int row = srow[k];
    // coupling rows (row >= nrows): right-hand side and dot entry 0, output in cpl
    const bool own = row >= 0 && row < nrows;
    rd_s[(k * R + c) * 2] = own ? rhs[(size_t)row * ld + c] : T(0);
    rd_s[(k * R + c) * 2 + 1] = (own && dotv != nullptr) ? dotv[(size_t)row * ld + c] : T(0);
    if (own)
      out[(size_t)row * ld + c] = sentinel_value<T>();
    else if (row >= nrows)
      cpl[(size_t)(row - nrows) * ld + c] = sentinel_value<T>();
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
template <typename T, int R>
size_t trsv_shmem_t(int nslots, bool compact) {
  return 64 + SlotLayout<T, R>::bytes(nslots, compact ? SlotLayout<T, R>::kCompact : 0);
}

size_t trsv_shmem_bytes(int nslots, bool fp32, int R, bool compact) {
  if (fp32) {
    switch (R) {
      case 1: return trsv_shmem_t<float, 1>(nslots, compact);
      case 8: return trsv_shmem_t<float, 8>(nslots, compact);
      default: return trsv_shmem_t<float, 16>(nslots, compact);
    }
  }
  switch (R) {
    case 1: return trsv_shmem_t<double, 1>(nslots, compact);
    case 8: return trsv_shmem_t<double, 8>(nslots, compact);
    default: return trsv_shmem_t<double, 16>(nslots, compact);
  }
}

// H column blocks of R columns each in one launch (H > 1: column-split kernel only; the
// blocks' groups must all be resident, which the caller has checked).
template <typename T, int R, int EP, int D>
static hipError_t launch_trsv_t(const TrsvSchedDev& S, const T* sval, const typename RowRec<T>::type* srinfo,
                                const T* rhs, T* out, T* cpl, const T* dotv, double* dot_out, int ld, const int* skip,
                                hipStream_t st, const TrsvTiming* tm, int H) {
  TrsvArgs a;
  a.grp_step_ptr = S.grp_step_ptr;
  a.grp_ep = S.grp_ep;
  a.grp_eoff = S.grp_eoff;
  a.grp_halo_ptr = S.grp_halo_ptr;
  a.halo_row = S.halo_row;
  a.halo_slot = S.halo_slot;
  a.halo_free = S.halo_free;
  a.srow = S.srow;
  a.ssrc = S.ssrc;
  a.done_count = S.done_count;
  a.err = S.err;
  a.partials = S.partials;
  a.ngroups = S.ngroups;
  a.nslots = S.nslots;
  a.nrows = S.nrows;
  a.ld = ld;
  a.cpl = cpl;
  a.ncpl = S.ncpl;
  T* rd_s = reinterpret_cast<T*>(S.rhs_s);
  T* dummy = reinterpret_cast<T*>(S.dummy);
  const int64_t nrow_slots = (int64_t)S.nsteps * kTrsvRPS;
  a.nrow_slots = nrow_slots;
  for (int h = 0; h < H; ++h)
    hipLaunchKernelGGL((k_trsv_gather_rhs<T, R>), dim3(1024), dim3(256), 0, st, nrow_slots, S.srow, rhs + h * R,
                       dotv ? dotv + h * R : nullptr, ld, rd_s + (size_t)h * nrow_slots * 2 * R, out + h * R,
                       cpl ? cpl + h * R : nullptr, S.nrows, skip);
  const size_t shmem = trsv_shmem_t<T, R>(S.nslots, H > 1);
  // R >= 8 and at most 8 entries per lane (coupled schedules, 2D and 3D): the columns split
  // over W = 2 compute wavefronts of RC = R / 2 columns each (every wave reads the step's
  // records, so fewer waves read fewer bytes; 4 waves of R / 4 columns measured 2-8 %
  // slower, 8 waves of 2 columns 3.5x slower), with a prefetch depth that keeps the step
  // buffers in 256 registers.  Rows with more entries per lane keep one compute wavefront.
  constexpr int RC = R / 2 > Vec16<T>::n ? R / 2 : Vec16<T>::n;
  constexpr int W = (R >= 8 && EP <= 8) ? R / RC : 0;
  constexpr int GC = RC / Vec16<T>::n;
  constexpr int DC = cols_depth(GC, EP);
  const void* fn;
  int threads;
  if constexpr (W > 0) {
    // two workgroups per CU (H > 1) need the compact slot padding
    fn = H > 1 ? (const void*)k_trsv_cols<T, R, EP, DC, W, SlotLayout<T, R>::kCompact>
               : (const void*)k_trsv_cols<T, R, EP, DC, W, 0>;
    threads = 64 * (W + 1);
  } else {
    if (H != 1) return hipErrorInvalidValue;
    fn = (const void*)k_trsv<T, R, EP, D>;
    threads = kTrsvThreads;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  if (e != hipSuccess) return e;
  const T* rd_sc = rd_s;
  int with_dot = dotv != nullptr ? 1 : 0;
  void* args[] = {&a, &sval, &srinfo, &rd_sc, &out, &dummy, &with_dot, &dot_out, &skip};
  if (tm && tm->before) (void)hipEventRecord(tm->before, st);
  // An ordinary launch: the host has checked that every group fits on the chip at once,
  // so all groups are dispatched together (a cooperative launch adds tens of microseconds
  // of queue synchronisation around the kernel and is not needed for that).
  e = hipLaunchKernel(fn, dim3(S.ngroups * H), dim3(threads), args, shmem, st);
  if (tm && tm->after) (void)hipEventRecord(tm->after, st);
  return e;
}

template <typename T, int R>
static hipError_t launch_trsv_r(const TrsvSchedDev& S, const T* sval, const typename RowRec<T>::type* srinfo,
                                const T* rhs, T* out, T* cpl, const T* dotv, double* dot_out, int ld, const int* skip,
                                hipStream_t st, const TrsvTiming* tm, int H) {
  switch (S.EP) {
    case 4: return launch_trsv_t<T, R, 4, batch_depth(R, 4, sizeof(T))>(S, sval, srinfo, rhs, out, cpl, dotv, dot_out, ld, skip, st, tm, H);
    case 8: return launch_trsv_t<T, R, 8, batch_depth(R, 8, sizeof(T))>(S, sval, srinfo, rhs, out, cpl, dotv, dot_out, ld, skip, st, tm, H);
    case 12: return launch_trsv_t<T, R, 12, batch_depth(R, 12, sizeof(T))>(S, sval, srinfo, rhs, out, cpl, dotv, dot_out, ld, skip, st, tm, H);
    case 16: return launch_trsv_t<T, R, 16, batch_depth(R, 16, sizeof(T))>(S, sval, srinfo, rhs, out, cpl, dotv, dot_out, ld, skip, st, tm, H);
  }
  return hipErrorInvalidValue;
}

// R columns in chunks of the widest width whose LDS slots fit (R, 8 or 1), one launch each;
// a 16-column batch whose 8-column blocks fit two workgroups per CU instead runs as one
// launch of two 8-column blocks side by side (each step then carries half the columns).
template <typename T>
static hipError_t launch_trsv_p(const TrsvSchedDev& S, const T* sval, const typename RowRec<T>::type* srinfo, int R,
                                const T* rhs, T* out, const T* dotv, double* dot_out, const int* skip, hipStream_t st,
                                const TrsvTiming* tm) {
  int dev = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  int Rc = R;
  while (Rc > 1 && (Rc > S.rmax || trsv_shmem_bytes(S.nslots, sizeof(T) == 4, Rc) + trsv_static_shmem(Rc) > (size_t)lds_max))
    Rc = Rc > 8 ? 8 : 1;
  if (R % Rc != 0) return hipErrorInvalidValue;
  int H = 1;
  if (Rc == 16 && S.EP <= 8) {
    int ncu = 0, lds_cu = 0;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e != hipSuccess) return e;
    const size_t lds8 = trsv_shmem_bytes(S.nslots, sizeof(T) == 4, 8, true) + trsv_static_shmem(8);
    // two workgroups of three wavefronts (at most 256 registers each) per CU
    const int per_cu = (int)std::min<size_t>(2, (size_t)lds_cu / lds8);
    if (per_cu >= 2 && 2 * S.ngroups <= per_cu * ncu) {
      Rc = 8;
      H = 2;
    }
  }
  // coupling rows' values: [ncpl][R] in the schedule's buffer (sized for the widest batch)
  T* cpl = reinterpret_cast<T*>(S.cpl);
  if (S.ncpl > 0 && (cpl == nullptr || R > kRMax)) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < R; c0 += Rc * H) {
    // timing events: before the first chunk, after the last
    TrsvTiming t;
    if (tm != nullptr) {
      t.before = c0 == 0 ? tm->before : nullptr;
      t.after = c0 + Rc * H >= R ? tm->after : nullptr;
    }
    const T* dv = dotv ? dotv + c0 : nullptr;
    double* dout = dot_out ? dot_out + c0 : nullptr;
    T* cc = cpl ? cpl + c0 : nullptr;
    switch (Rc) {
      case 1: e = launch_trsv_r<T, 1>(S, sval, srinfo, rhs + c0, out + c0, cc, dv, dout, R, skip, st, &t, 1); break;
      case 8: e = launch_trsv_r<T, 8>(S, sval, srinfo, rhs + c0, out + c0, cc, dv, dout, R, skip, st, &t, H); break;
      case 16: e = launch_trsv_r<T, 16>(S, sval, srinfo, rhs + c0, out + c0, cc, dv, dout, R, skip, st, &t, 1); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trsv(const TrsvSchedDev& S, bool fp32, int R, const void* rhs, void* out, const void* dotv,
                       double* dot_out, const int* skip, hipStream_t st, const TrsvTiming* tm) {
  if (R == 1 && S.fast.ok) {
    if (fp32)
      return launch_trsv_fast<float>(S, (const float*)rhs, (float*)out, (const float*)dotv, dot_out, skip, st, tm);
    return launch_trsv_fast<double>(S, (const double*)rhs, (double*)out, (const double*)dotv, dot_out, skip, st, tm);
  }
  if (fp32)
    return launch_trsv_p<float>(S, S.sval32, S.srinfo32, R, (const float*)rhs, (float*)out, (const float*)dotv,
                                dot_out, skip, st, tm);
  return launch_trsv_p<double>(S, S.sval, S.srinfo, R, (const double*)rhs, (double*)out, (const double*)dotv, dot_out,
                               skip, st, tm);
}

// Factor values into schedule order and reciprocal diagonals into the row records.
__global__ void k_trsv_gather(const int64_t* __restrict__ perm, int64_t n, const double* __restrict__ Lval,
                              double* __restrict__ out, float* __restrict__ out32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[i];
    const double v = p >= 0 ? Lval[p] : (p == kTrsvValOne ? 1.0 : 0.0);
    out[i] = v;
    out32[i] = (float)v;
  }
}

__global__ void k_trsv_gather_dinv(const int64_t* __restrict__ dsrc, int64_t n, const double* __restrict__ Lval,
                                   TrsvRow64* __restrict__ ri, TrsvRow32* __restrict__ ri32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = dsrc[i];
    ri[i].dinv = p >= 0 ? 1.0 / Lval[p] : (p == kTrsvValMinusOne ? -1.0 : 0.0);
    ri32[i].dinv = p >= 0 ? 1.0f / (float)Lval[p] : (p == kTrsvValMinusOne ? -1.0f : 0.0f);
  }
}

hipError_t launch_trsv_gather(const TrsvSchedDev& S, const double* Lval, hipStream_t st) {
  const int64_t ne = S.nent;
  const int64_t nd = (int64_t)S.nsteps * kTrsvRPS;
  hipLaunchKernelGGL(k_trsv_gather, dim3(1024), dim3(256), 0, st, S.vperm, ne, Lval, S.sval, S.sval32);
  hipLaunchKernelGGL(k_trsv_gather_dinv, dim3(256), dim3(256), 0, st, S.dsrc, nd, Lval, S.srinfo, S.srinfo32);
  if (S.fast.ok)
    hipLaunchKernelGGL(k_fast_gather_static, dim3(1024), dim3(256), 0, st, (int64_t)S.fast.nsteps, S.fast.step_val64,
                       S.fast.step_val32, S.fast.step_ep, S.fast.vperm, S.fast.dsrc, Lval, S.fast.blk64, S.fast.blk32);
  return hipGetLastError();
}

}  // namespace stk

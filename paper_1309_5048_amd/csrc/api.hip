// C ABI of libstokes.so (declared in include/stokes.h): problem setup, the MINRES
// drivers (FP64, mixed FP32/FP64 refinement, batched, adjoint) and small utilities.
// Host code only orchestrates; every arithmetic step of the method runs in the HIP
// kernels of this library.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>

#include "stokes.h"
#include "stokes_internal.h"

using namespace stk;

namespace {

// ---------------------------------------------------------------------------
// Small kernels used only by the orchestration
// ---------------------------------------------------------------------------
__global__ void k_gather_diag(int64_t n, const int32_t* __restrict__ Lrowptr, const int64_t* __restrict__ Lsrc,
                              const double* __restrict__ val, double* __restrict__ diagA) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    diagA[i] = val[Lsrc[Lrowptr[i + 1] - 1]];
}

// pressure-weighted column sums: out[c] = sum_k wt[k] * x[(off+k)*R + c] (wt = nullptr: plain sum)
template <int R>
__global__ __launch_bounds__(kVT) void k_pdot(int64_t np, int64_t off, const double* __restrict__ wt,
                                              const double* __restrict__ x, double* partials, unsigned int* counter,
                                              double* out) {
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t k = blockIdx.x * (int64_t)kVT + threadIdx.x; k < np; k += (int64_t)gridDim.x * kVT) {
    const double wv = wt ? wt[k] : 1.0;
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] += wv * x[(size_t)(off + k) * R + c];
  }
  reduce_last<R>(acc, partials, counter, [&](int k, double v) { out[k] = v; });
}

// M^{-1}-weighted squares of the pressure part (2 nu r^2 / diagQ) and, with diagA, of the
// velocity part (r^2 / diagA): out[c] = pressure part, out[R+c] = velocity part.
template <int R>
__global__ __launch_bounds__(kVT) void k_diag_wsq(int64_t n_u, int64_t n, const double* __restrict__ r,
                                                  const double* __restrict__ diagQ, const double* __restrict__ diagA,
                                                  double two_nu, double* partials, unsigned int* counter, double* out) {
  double acc[2 * R];
#pragma unroll
  for (int c = 0; c < 2 * R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVT) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double rv = r[(size_t)i * R + c];
      if (i >= n_u) acc[c] += two_nu * rv * rv / diagQ[i - n_u];
      else if (diagA) acc[R + c] += rv * rv / diagA[i];
    }
  }
  reduce_last<2 * R>(acc, partials, counter, [&](int k, double v) { out[k] = v; });
}

// b_p -= w * s[c] / w1 (adjoint right-hand side P^T g_p)
template <int R>
__global__ void k_sub_w(int64_t n_u, int64_t np, double* __restrict__ b, const double* __restrict__ w,
                        const double* __restrict__ s, double w1) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < np; k += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < R; ++c) b[(size_t)(n_u + k) * R + c] -= w[k] * s[c] / w1;
}

// z = M^{-1} r for the diagonal blocks (pressure always, velocity with diagA), R = 1
__global__ void k_apply_diag(int64_t n_u, int64_t n, const double* __restrict__ r, double* __restrict__ z,
                             const double* __restrict__ diagQ, const double* __restrict__ diagA, double two_nu) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i >= n_u) z[i] = two_nu * r[i] / diagQ[i - n_u];
    else if (diagA) z[i] = r[i] / diagA[i];
  }
}

// A part of the saddle values (velocity rows, columns < n_u) scaled by s
__global__ void k_scale_A(int64_t n_u, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ aend,
                          double* __restrict__ val, double s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * blockDim.x)
    for (int32_t k = rowptr[i]; k < aend[i]; ++k) val[k] *= s;
}

template <typename T>
__global__ void k_fill(int64_t n, T* __restrict__ a, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] = v;
}

#define R_SWITCH(R_, ...)                                   \
  switch (R_) {                                             \
    case 1: { constexpr int RR = 1; __VA_ARGS__; break; }   \
    case 8: { constexpr int RR = 8; __VA_ARGS__; break; }   \
    case 16: { constexpr int RR = 16; __VA_ARGS__; break; } \
    default: break;                                         \
  }

// ---------------------------------------------------------------------------
// Workspace of stokes_solve_noalloc: a file-scope device array, one copy per GPU, held
// until the process ends.  Host code never passes the array's name to a kernel (in host
// code it is only a stand-in for the symbol): stokes_setup looks up the address of the
// current device's copy with hipGetSymbolAddress, and every use goes through that pointer.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = size_t(64) << 20;  // 64 MiB
constexpr int kNoAllocVectors = 10;                  // MINRES vectors v, z, w (x2), x, q, b, y
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// ---------------------------------------------------------------------------
// Device buffer helpers
// ---------------------------------------------------------------------------
struct DevAlloc {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <typename T>
  T* get(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      err = e;
      return nullptr;
    }
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <typename T>
  T* upload(const std::vector<T>& v, hipStream_t st) {
    T* p = get<T>(v.size());
    if (p && !v.empty()) {
      hipError_t e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
      if (e != hipSuccess) err = e;
    }
    return p;
  }
  void release() {
    for (void* p : ptrs) hipFree(p);
    ptrs.clear();
  }
};

struct SchedPair {
  TrsvSchedDev fwd, bwd;
  int strip = 0;
  int rmax64 = 0, rmax32 = 0;
};

// An IC(0) factor with its triangular-solve schedules: the pattern (host), the factor
// values (device), the dependency levels of both solves, and a strip partition of the
// rows by height.
struct FactorSched {
  const LowerPattern* L = nullptr;
  int64_t n = 0;
  const double* Lval = nullptr;
  const std::vector<int32_t>* lev_fwd = nullptr;
  std::vector<int32_t>* lev_bwd = nullptr;
  std::function<void(int, std::vector<int32_t>&, int*)> groups;
  // row blocks solved one after another (offsets; the velocity components of A's factor):
  // the solves then take each row's dependencies on earlier blocks as coupling values from
  // `helpers` extra groups per (strip, source block); fewer than two blocks or no helpers:
  // off
  std::vector<int64_t> blocks;
  int helpers = 0;
  std::vector<std::unique_ptr<SchedPair>> scheds;
};

// Workspace of one (R, precision) combination; vectors interleaved [row][R].
struct Work {
  int R = 0;
  bool fp32 = false;
  void *v[2] = {nullptr, nullptr}, *z[2] = {nullptr, nullptr}, *w[2] = {nullptr, nullptr};
  void *x = nullptr, *q = nullptr, *b = nullptr, *y = nullptr;
  void *pr = nullptr, *pp = nullptr, *pq = nullptr, *pz = nullptr;  // inner PCG
  void *qr = nullptr, *qp = nullptr, *qq = nullptr, *qz = nullptr;  // pressure-block PCG
  void* qy = nullptr;  // pressure-block IC(0): between the two triangular solves
  void *xr = nullptr, *br = nullptr;  // refinement: accumulated solution, original rhs (FP64)
};

}  // namespace

struct stokes_problem {
  Spaces S;
  double nu = 1.0, cpen = 0.0;
  hipStream_t stream = nullptr;
  std::string err;
  SaddlePattern P;
  LowerPattern L;
  std::vector<int32_t> level_ptr;
  int nlev_fwd = 0;
  int64_t nnz = 0, nnzL = 0;
  DevAlloc mem;  // everything owned by the problem
  int32_t *rowptr = nullptr, *col = nullptr, *aend = nullptr;
  RowSplit rs_full, rs_A;  // row ranges of the row kernels: all rows / A part of velocity rows
  std::vector<int32_t> split_full_h, split_A_h;  // host copies (kept alive for the async upload)
  double* val = nullptr;
  float* val32 = nullptr;
  double *diagQ = nullptr, *w = nullptr, *diagA = nullptr;
  // coefficients of the constant function in the pressure space: null on the identity map
  // (all ones); Q^{-1} w on a mapped domain (phi = phihat / J)
  double* kappa = nullptr;
  double w1 = 1.0;  // w . kappa = |Omega|
  int32_t *Lrowptr = nullptr, *Lcol = nullptr, *level_rows = nullptr;
  int64_t* Lsrc = nullptr;
  double* Lval = nullptr;
  int* flag = nullptr;
  int ic_shift_steps = 0;
  FactorSched fsA;  // IC(0) of A and its schedules
  MrScalars mr;
  PcgScalars pcg;
  // pressure-block CG (PCG(A,Q)): Q in CSR, its row ranges, FP32 values, scalars
  int32_t *Qrowptr = nullptr, *Qcol = nullptr;
  double* Qval = nullptr;
  float* Qval32 = nullptr;
  RowSplit rs_Q;
  std::vector<int32_t> Qrowptr_h, Qcol_h, split_Q_h;
  PcgScalars pcgQ;
  // IC(0) of Q (IC(0)-PCG on the pressure block): lower pattern, values, levels, schedules
  LowerPattern LQ;
  std::vector<int32_t> levQ_fwd, levQ_bwd;
  int32_t *LQrowptr = nullptr, *LQcol = nullptr;
  int64_t* LQsrc = nullptr;
  double* LQval = nullptr;
  FactorSched fsQ;
  // inner CG iterations the last application needed, per velocity preconditioner and for
  // the pressure block (PCG(A,Q), Ideal(A,Q)): the first chunk queued before the host
  // reads the done flag
  int pcg_expect[8] = {4, 4, 4, 4, 4, 4, 4, 4}, pcgq_expect[3] = {4, 4, 4};
  double* scratch = nullptr;  // [64] small host-visible results
  double* partials = nullptr;
  unsigned int* counter = nullptr;
  std::map<int, Work> work;
  // saddle product with non-temporal entry loads: only while the two FP64 triangular-solve
  // schedules fit the 256 MB last-level cache (2 x 102 MB at N = 256, k' = 2), which the
  // product's entries would otherwise evict every iteration
  bool spmv_nt = true;
  double inner_tol = 1e-2;
  double refine_tol = 1e-4;
  int restarts = 0;  // inner-CG preconditioners: 0 = one MINRES run, else at most this many cycles
  int maxit_outer = 20000, maxit_inner = 200;
  int check_every = 8;
  double setup_ms = 0.0;
  size_t lds_max = 65536;
  size_t lds_per_cu = 65536;
  int num_cu = 0;
  std::vector<int32_t> lev_fwd, lev_bwd;  // dependency levels of the two solves
  // live kernel timing (HIP events on the problem's stream), enabled by stokes_profile
  bool prof_on = false;
  std::vector<TrsvTiming> prof_pool;
  std::vector<int> prof_cat;
  size_t prof_used = 0;
  double prof_ms[5] = {0, 0, 0, 0, 0};
  int64_t prof_cnt[5] = {0, 0, 0, 0, 0};
  // convergence polling: two pinned host flags and their completion events
  int* hflag = nullptr;
  hipEvent_t flag_ev[2] = {nullptr, nullptr};
  // the same for the inner CG loops
  int* pcg_hflag = nullptr;
  hipEvent_t pcg_ev[2] = {nullptr, nullptr};
  // timing events of stokes_solve_noalloc, created at setup
  hipEvent_t noalloc_ev[2] = {nullptr, nullptr};
  // this device's copy of the stokes_solve_noalloc workspace (looked up at setup)
  void* noalloc_ws = nullptr;
  ~stokes_problem() {
    for (auto& e : noalloc_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& t : prof_pool) {
      (void)hipEventDestroy(t.before);
      (void)hipEventDestroy(t.after);
    }
    for (auto& e : flag_ev)
      if (e) (void)hipEventDestroy(e);
    if (hflag) (void)hipHostFree(hflag);
    for (auto& e : pcg_ev)
      if (e) (void)hipEventDestroy(e);
    if (pcg_hflag) (void)hipHostFree(pcg_hflag);
    mem.release();
  }
};

namespace {

int fail(stokes_problem* pb, int code, const std::string& msg) {
  if (pb) pb->err = msg;
  return code;
}

int fail_hip(stokes_problem* pb, hipError_t e, const char* what, int line) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at api.hip:%d", int(e), hipGetErrorString(e), what, line);
  if (pb) pb->err = buf;
  return e == hipErrorOutOfMemory ? STOKES_ENOMEM : STOKES_EHIP;
}

#define CK(...)                                                          \
  do {                                                                   \
    hipError_t _e = (__VA_ARGS__);                                       \
    if (_e != hipSuccess) return fail_hip(pb, _e, #__VA_ARGS__, __LINE__); \
  } while (0)

// Event pair for one timed launch of category cat (0 saddle SpMV, 1 forward solve,
// 2 backward solve, 3 Lanczos update, 4 Givens/w/x update); null when profiling is off.
const TrsvTiming* prof_take(stokes_problem* pb, int cat) {
  if (!pb->prof_on) return nullptr;
  if (pb->prof_used == pb->prof_pool.size()) {
    TrsvTiming t;
    if (hipEventCreate(&t.before) != hipSuccess || hipEventCreate(&t.after) != hipSuccess) return nullptr;
    pb->prof_pool.push_back(t);
    pb->prof_cat.push_back(0);
  }
  pb->prof_cat[pb->prof_used] = cat;
  return &pb->prof_pool[pb->prof_used++];
}

// Accumulate the elapsed times of the recorded pairs that have completed; pairs still in
// flight stay in the pool for a later call.
void prof_flush(stokes_problem* pb) {
  size_t keep = 0;
  for (size_t k = 0; k < pb->prof_used; ++k) {
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, pb->prof_pool[k].before, pb->prof_pool[k].after);
    if (e == hipErrorNotReady) {
      std::swap(pb->prof_pool[keep], pb->prof_pool[k]);
      std::swap(pb->prof_cat[keep], pb->prof_cat[k]);
      ++keep;
      continue;
    }
    if (e == hipSuccess) {
      pb->prof_ms[pb->prof_cat[k]] += ms;
      pb->prof_cnt[pb->prof_cat[k]] += 1;
    }
  }
  pb->prof_used = keep;
}

#define PROF_BEGIN(cat)                                   \
  const TrsvTiming* _pt = prof_take(pb, cat);             \
  if (_pt) (void)hipEventRecord(_pt->before, pb->stream);
#define PROF_END() \
  if (_pt) (void)hipEventRecord(_pt->after, pb->stream);

// Single-column layout of a schedule H (see TrsvFastDev); H may have coupling rows and
// helper groups.  Returns 0 and leaves F.ok false when a group needs more than 8 entries per
// lane (the general kernel then serves R = 1).
int build_fast_layout(stokes_problem* pb, const TrsvSchedHost& H, TrsvSchedDev& D, int64_t nrows, int64_t nnzL) {
  TrsvFastDev& F = D.fast;
  hipStream_t st = pb->stream;
  DevAlloc& m = pb->mem;
  const int G = H.ngroups, RPS = kTrsvRPS, E = H.E;
  if (nrows + H.ncpl >= (int64_t(1) << 31)) return 0;
  if (nrows * 8 >= (int64_t(1) << 31) || nnzL >= (int64_t(1) << 31)) return 0;
  std::vector<int32_t> gsp(G + 1, 0), gnp(G, 0), gep(G, 4);
  std::vector<int64_t> gb64(G + 1, 0), gb32(G + 1, 0);
  int64_t off64 = 0, off32 = 0;
  for (int g = 0; g < G; ++g) {
    const int s0 = H.grp_step_ptr[g], s1 = H.grp_step_ptr[g + 1];
    int eg = 0;
    for (int s = s0; s < s1; ++s)
      for (int e = 0; e < E; ++e)
        for (int l = 0; l < 64; ++l)
          if (H.ent_perm[(size_t(s) * E + e) * 64 + l] != -1) eg = std::max(eg, e + 1);
    if (eg > 8) return 0;
    gep[g] = eg <= 4 ? 4 : 8;
    const int nreal = s1 - s0, dg = fast_depth(gep[g]);
    gnp[g] = nreal > 0 ? (nreal + dg - 1) / dg * dg : 0;
    const int alloc = nreal > 0 ? gnp[g] + dg : 0;
    gsp[g + 1] = gsp[g] + alloc;
    gb64[g] = off64;
    gb32[g] = off32;
    off64 += int64_t(alloc) * fast_block_bytes<double>(gep[g]);
    off32 += int64_t(alloc) * fast_block_bytes<float>(gep[g]);
  }
  gb64[G] = off64;
  gb32[G] = off32;
  F.bytes64 = off64;
  if (off64 >= (int64_t(1) << 31)) return 0;  // block offsets of a group must fit 32 bits
  const int64_t T = gsp[G];
  std::vector<unsigned char> b64(size_t(off64), 0), b32(size_t(off32), 0);
  std::vector<int64_t> sv64(T), sv32(T);
  std::vector<int32_t> sep(T), vperm(size_t(T) * 64 * 8, -1), dsrc(size_t(T) * RPS, -1), srow2(size_t(T) * RPS, 0);
  for (int g = 0; g < G; ++g) {
    const int s0 = H.grp_step_ptr[g], nreal = H.grp_step_ptr[g + 1] - s0, ep = gep[g];
    const int sb64 = fast_block_bytes<double>(ep), sb32 = fast_block_bytes<float>(ep);
    for (int j = 0; j < gsp[g + 1] - gsp[g]; ++j) {
      const int64_t t = gsp[g] + j;
      const int s = s0 + std::min(j, nreal - 1);
      const bool repeat_step = j >= nreal;
      unsigned char* p64 = b64.data() + gb64[g] + int64_t(j) * sb64;
      unsigned char* p32 = b32.data() + gb32[g] + int64_t(j) * sb32;
      sv64[t] = gb64[g] + int64_t(j) * sb64 + kFastHdr + 64 * ep * 4;
      sv32[t] = gb32[g] + int64_t(j) * sb32 + kFastHdr + 64 * ep * 4;
      sep[t] = ep;
      const int32_t need = H.step_halo_need[s];
      if (need > kFastMaxField) return 0;  // the general kernel serves this schedule
      const int32_t row0 = H.srow[size_t(s) * RPS];
      if (row0 < 0) return fail(pb, STOKES_EINVAL, "triangular-solve step without rows");
      for (int rr = 0; rr < RPS; ++rr) {
        const int32_t row = H.srow[size_t(s) * RPS + rr];
        const int src = row >= 0 ? rr : 0;  // missing rows repeat row 0
        const int32_t srow = H.srow[size_t(s) * RPS + src];
        srow2[size_t(t) * RPS + rr] = (row >= 0 && !repeat_step) ? srow : ~srow;
        dsrc[size_t(t) * RPS + rr] = int32_t(H.sdiag_src[size_t(s) * RPS + src]);
        const int32_t slot = H.sslot[size_t(s) * RPS + src] > 0 ? H.sslot[size_t(s) * RPS + src] : H.nslots;
        // coupling rows are stored apart, from row nrows on (a group holds one kind only)
        if ((srow >= nrows) != (H.grp_cpl[g] != 0))
          return fail(pb, STOKES_EINVAL, "coupling row outside a helper group");
        const int32_t orow = int32_t(srow >= nrows ? srow - nrows : srow);
        if (64 + slot * 8 > kFastMaxField) return 0;
        FastRec64 r64{0.0, uint32_t(64 + slot * 8) | (uint32_t(need) << 16), int32_t(orow * 8)};
        FastRec32 r32{0.0f, int32_t(64 + slot * 4), int32_t(orow * 4), need};
        std::memcpy(p64 + rr * 16, &r64, 16);
        std::memcpy(p32 + rr * 16, &r32, 16);
        for (int q = 0; q < kTrsvG; ++q) {
          const int lane = rr * kTrsvG + q, lsrc = src * kTrsvG + q;
          for (int e = 0; e < ep; ++e) {
            int64_t vp = -1;
            int32_t sl = 0;
            if (e < E) {
              vp = H.ent_perm[(size_t(s) * E + e) * 64 + lsrc];
              sl = H.ent_src[(size_t(s) * E + e) * 64 + lsrc];
            }
            vperm[(size_t(t) * 64 + lane) * 8 + e] = int32_t(vp);
            const uint32_t a64 = uint32_t(64 + sl * 8), a32 = uint32_t(64 + sl * 4);
            std::memcpy(p64 + kFastHdr + (lane * ep + e) * 4, &a64, 4);
            std::memcpy(p32 + kFastHdr + (lane * ep + e) * 4, &a32, 4);
          }
        }
      }
    }
  }
  F.nsteps = int(T);
  F.grp_step_ptr = m.upload(gsp, st);
  F.grp_npad = m.upload(gnp, st);
  F.grp_ep = m.upload(gep, st);
  F.grp_blk64 = m.upload(gb64, st);
  F.grp_blk32 = m.upload(gb32, st);
  F.blk64 = m.upload(b64, st);
  F.blk32 = m.upload(b32, st);
  F.step_val64 = m.upload(sv64, st);
  F.step_val32 = m.upload(sv32, st);
  F.step_ep = m.upload(sep, st);
  F.vperm = m.upload(vperm, st);
  F.dsrc = m.upload(dsrc, st);
  F.srow2 = m.upload(srow2, st);
  F.dyn = m.get<double>(size_t(T) * RPS * 2);
  F.ngroups = G;
  F.nslots = H.nslots;
  F.nrows = int(nrows);
  F.ncpl = int(H.ncpl);
  F.grp_halo_ptr = m.upload(H.grp_halo_ptr, st);
  F.halo_row = m.upload(H.halo_row, st);
  F.halo_slot = m.upload(H.halo_slot, st);
  F.halo_free = m.upload(H.halo_free, st);
  F.grp_cpl = m.upload(H.grp_cpl, st);
  F.cpl = m.get<double>(size_t(std::max<int64_t>(1, H.ncpl)));
  F.done_count = m.get<unsigned int>(1);
  F.partials = m.get<double>(size_t(G));
  if (m.err != hipSuccess) return fail_hip(pb, m.err, "single-column schedule upload", __LINE__);
  CK(hipMemsetAsync(F.done_count, 0, sizeof(unsigned int), st));
  CK(hipStreamSynchronize(st));  // the host vectors must outlive the copies
  F.ok = true;
  return 0;
}

// Device form of a schedule of the factor Lval (nrows rows, nnzL entries; rows from nrows on
// are coupling rows).
int upload_schedule(stokes_problem* pb, const TrsvSchedHost& H, TrsvSchedDev& D, int rmax, int64_t nrows,
                    int64_t nnzL, const double* Lval) {
  hipStream_t st = pb->stream;
  DevAlloc& m = pb->mem;
  D.ngroups = H.ngroups;
  D.nsteps = H.nsteps;
  D.E = H.E;
  D.nlevels = H.nlevels;
  D.nslots = H.nslots;
  D.nrows = int(nrows);
  const size_t ns = size_t(H.nsteps);
  // per-lane records: values (via a permutation into L) and 32-bit slot ids, EP per lane
  // for each group (its widest row over kTrsvG lanes, a multiple of 4; 4 or the largest
  // of the schedule, the two widths the kernels take), steps of a group contiguous
  std::vector<int32_t> gep(H.ngroups, 4);
  std::vector<int64_t> geoff(H.ngroups + 1, 0);
  D.EP = 4;
  for (int g = 0; g < H.ngroups; ++g) {
    int eg = 1;
    for (int s = H.grp_step_ptr[g]; s < H.grp_step_ptr[g + 1]; ++s)
      for (int e = 0; e < H.E; ++e)
        for (int l = 0; l < 64; ++l)
          if (H.ent_perm[(size_t(s) * H.E + e) * 64 + l] != -1) eg = std::max(eg, e + 1);
    gep[g] = (eg + 3) / 4 * 4;
    D.EP = std::max(D.EP, gep[g]);
  }
  for (int g = 0; g < H.ngroups; ++g) {
    if (gep[g] > 4) gep[g] = D.EP;
    geoff[g + 1] = geoff[g] + int64_t(H.grp_step_ptr[g + 1] - H.grp_step_ptr[g]) * 64 * gep[g];
  }
  const size_t nent = size_t(geoff[H.ngroups]);
  std::vector<int64_t> vperm(nent, -1);
  std::vector<uint32_t> ssrc(nent, 0);
  for (int g = 0; g < H.ngroups; ++g)
    for (int s = H.grp_step_ptr[g]; s < H.grp_step_ptr[g + 1]; ++s)
      for (int e = 0; e < std::min(H.E, gep[g]); ++e)
        for (int l = 0; l < 64; ++l) {
          const size_t from = (size_t(s) * H.E + e) * 64 + l;
          const size_t to = size_t(geoff[g]) + (size_t(s - H.grp_step_ptr[g]) * 64 + l) * gep[g] + e;
          vperm[to] = H.ent_perm[from];
          ssrc[to] = uint32_t(H.ent_src[from]);
        }
  D.nent = int64_t(nent);
  std::vector<TrsvRow64> ri(ns * kTrsvRPS);
  std::vector<TrsvRow32> ri32(ns * kTrsvRPS);
  for (size_t k = 0; k < ns * kTrsvRPS; ++k) {
    const int32_t need = H.step_halo_need[k / kTrsvRPS];
    // rows whose value no later step reads write to the dummy slot nslots
    const int32_t slot = H.sslot[k] > 0 ? H.sslot[k] : H.nslots;
    ri[k].dinv = 0.0;
    ri[k].slot = slot;
    ri[k].need = need;
    ri32[k].dinv = 0.0f;
    ri32[k].slot = slot;
    ri32[k].need = need;
    ri32[k].pad = 0;
  }
  std::vector<TrsvStep> sst(ns);
  for (size_t s = 0; s < ns; ++s) sst[s] = TrsvStep{H.step_level[s], H.step_publish[s], H.step_halo_need[s], 0};
  D.grp_step_ptr = m.upload(H.grp_step_ptr, st);
  D.grp_ep = m.upload(gep, st);
  D.grp_eoff = m.upload(geoff, st);
  D.grp_halo_ptr = m.upload(H.grp_halo_ptr, st);
  D.halo_row = m.upload(H.halo_row, st);
  D.halo_grp = m.upload(H.halo_grp, st);
  D.halo_lvl = m.upload(H.halo_lvl, st);
  D.halo_slot = m.upload(H.halo_slot, st);
  D.halo_free = m.upload(H.halo_free, st);
  D.srow = m.upload(H.srow, st);
  D.ssrc = m.upload(ssrc, st);
  D.vperm = m.upload(vperm, st);
  D.dsrc = m.upload(H.sdiag_src, st);
  D.sstep = m.upload(sst, st);
  D.srinfo = m.upload(ri, st);
  D.srinfo32 = m.upload(ri32, st);
  D.sval = m.get<double>(vperm.size());
  D.sval32 = m.get<float>(vperm.size());
  D.rhs_s = m.get<double>(H.srow.size() * 2 * std::max(1, rmax));
  D.dummy = m.get<double>((size_t)kTrsvDummyGroups * 64);
  D.progress = m.get<unsigned long long>(H.ngroups);
  D.epoch = m.get<unsigned long long>(1);
  D.done_count = m.get<unsigned int>(2);  // one ticket per column block of a launch
  D.err = m.get<int>(1);
  D.partials = m.get<double>(size_t(H.ngroups) * kRMax);
  D.ncpl = int(H.ncpl);
  D.cpl = H.ncpl > 0 ? m.get<double>(size_t(H.ncpl) * kRMax) : nullptr;
  D.rmax = rmax;
  if (m.err != hipSuccess) return fail_hip(pb, m.err, "schedule upload", __LINE__);
  CK(hipMemsetAsync(D.progress, 0, sizeof(unsigned long long) * H.ngroups, st));
  CK(hipMemsetAsync(D.epoch, 0, sizeof(unsigned long long), st));
  CK(hipMemsetAsync(D.done_count, 0, 2 * sizeof(unsigned int), st));
  CK(hipMemsetAsync(D.err, 0, sizeof(int), st));
  CK(hipStreamSynchronize(st));  // host vectors must outlive the asynchronous copies
  int rc = build_fast_layout(pb, H, D, nrows, nnzL);
  if (rc) return rc;
  CK(launch_trsv_gather(D, Lval, st));
  CK(hipStreamSynchronize(st));
  return 0;
}

// Largest R in {16, 8, 1} whose LDS footprint fits.
int fit_rmax(const stokes_problem* pb, int nslots, bool fp32) {
  const int rs[3] = {16, 8, 1};
  for (int r : rs)
    if (trsv_shmem_bytes(nslots, fp32, r) + trsv_static_shmem(r) <= pb->lds_max) return r;
  return 0;
}

// Largest rows-per-level of any (group, level) of a strip partition, over both solves.
int max_rows_per_level(const FactorSched& fs, const std::vector<int32_t>& group_of, int ngroups) {
  int worst = 0;
  for (int dir = 0; dir < 2; ++dir) {
    const auto& lev = dir == 0 ? *fs.lev_fwd : *fs.lev_bwd;
    int nl = 0;
    for (int32_t l : lev) nl = std::max(nl, l + 1);
    std::vector<int32_t> cnt(size_t(ngroups) * nl, 0);
    for (int64_t i = 0; i < fs.n; ++i) worst = std::max(worst, ++cnt[size_t(group_of[i]) * nl + lev[i]]);
  }
  return worst;
}

// Backward dependency levels: row i after every j > i with L_ji != 0.
void backward_levels(const LowerPattern& L, int64_t n, std::vector<int32_t>& lev) {
  lev.assign(n, 0);
  for (int64_t j = n - 1; j >= 0; --j) {
    const int lj = lev[j];
    for (int32_t k = L.rowptr[j]; k < L.rowptr[j + 1] - 1; ++k) {
      int32_t& li = lev[L.col[k]];
      li = std::max(li, lj + 1);
    }
  }
}

// Schedule pair usable for R columns in the given precision (built on first use).  The
// strip height is the largest that keeps one step per level (<= kTrsvRPS rows of a level
// per group), reduced further while the LDS window does not fit R columns or the groups
// cannot all be resident at once.
int make_schedule(stokes_problem* pb, FactorSched& fs, bool fp32, SchedPair** out) {
  for (auto& sp : fs.scheds)
    if ((fp32 ? sp->rmax32 : sp->rmax64) >= 1) {
      *out = sp.get();
      return 0;
    }
  if (fs.lev_bwd->empty()) backward_levels(*fs.L, fs.n, *fs.lev_bwd);
  const int strips[8] = {32, 16, 8, 4, 2, 1, 0, 0};
  int first = 0;
  for (int si = 0; strips[si] > 0; ++si) {
    std::vector<int32_t> group_of;
    int ngroups = 0;
    fs.groups(strips[si], group_of, &ngroups);
    if (max_rows_per_level(fs, group_of, ngroups) <= kTrsvRPS) {
      first = si;
      break;
    }
    first = si;
  }
  for (int si = first; strips[si] > 0; ++si) {
    const int strip = strips[si];
    bool exists = false;
    for (auto& sp : fs.scheds) exists |= (sp->strip == strip);
    if (exists) continue;
    std::vector<int32_t> group_of;
    int ngroups = 0;
    fs.groups(strip, group_of, &ngroups);
    std::string e;
    // all groups of a solve must be resident together (they wait on each other)
    auto fits = [&](const TrsvSchedHost& hf, const TrsvSchedHost& hb, SchedPair& sp) {
      const int nsl = std::max(hf.nslots, hb.nslots), ng = std::max(hf.ngroups, hb.ngroups);
      sp.rmax64 = fit_rmax(pb, nsl, false);
      sp.rmax32 = fit_rmax(pb, nsl, true);
      auto resident = [&](int r, bool f32) {
        if (r == 0) return 0;
        const size_t sh = trsv_shmem_bytes(nsl, f32, r);
        int per_cu = int(std::max<size_t>(1, std::min<size_t>(8, pb->lds_per_cu / std::max<size_t>(sh, 1))));
        // the batched kernels' blocks (up to five wavefronts of up to 256 registers) are
        // counted once per CU
        if (r >= 8) per_cu = 1;
        if (ng <= per_cu * pb->num_cu) return r;
        return (r >= 8 && ng <= pb->num_cu * 8) ? 1 : 0;  // then single columns only
      };
      sp.rmax64 = resident(sp.rmax64, false);
      sp.rmax32 = resident(sp.rmax32, true);
      return sp.rmax64 > 0 || sp.rmax32 > 0;
    };
    auto sp = std::make_unique<SchedPair>();
    sp->strip = strip;
    // Candidates: with coupling rows where the factor has row blocks (helpers per strip and
    // source block, then one), then the plain schedules.  The first whose batch width is
    // the widest any candidate allows is taken: more helpers shorten the chains of single
    // solves, but batched solves need every group resident with its R columns of slots.
    TrsvSchedHost hf, hb;
    int best = -1;
    {
      std::vector<int> hs;
      if (fs.blocks.size() > 2)
        for (int h = fs.helpers; h >= 1; h = h > 1 ? 1 : 0) hs.push_back(h);
      hs.push_back(0);  // plain
      int best_r = 0;
      for (size_t ci = 0; ci < hs.size(); ++ci) {
        TrsvSchedHost cf, cb;
        SchedPair t;
        const bool built =
            hs[ci] > 0
                ? build_trsv_schedule_coupled(*fs.L, fs.n, +1, fs.blocks, hs[ci], group_of, ngroups, cf, e) &&
                      build_trsv_schedule_coupled(*fs.L, fs.n, -1, fs.blocks, hs[ci], group_of, ngroups, cb, e)
                : build_trsv_schedule(*fs.L, fs.n, +1, group_of, ngroups, cf, e) &&
                      build_trsv_schedule(*fs.L, fs.n, -1, group_of, ngroups, cb, e);
        if (!built) {
          if (hs[ci] == 0) return fail(pb, STOKES_EINVAL, e);
          continue;
        }
        if (!fits(cf, cb, t)) continue;
        const int r = std::max(t.rmax64, t.rmax32);
        if (r > best_r) {
          best_r = r;
          best = int(ci);
          hf = std::move(cf);
          hb = std::move(cb);
          sp->rmax64 = t.rmax64;
          sp->rmax32 = t.rmax32;
        }
        if (best_r >= kRMax) break;  // no candidate can do better
      }
    }
    if (best < 0) continue;
    const int64_t nnzL = int64_t(fs.L->col.size());
    int rc = upload_schedule(pb, hf, sp->fwd, std::max(sp->rmax64, sp->rmax32), fs.n, nnzL, fs.Lval);
    if (rc) return rc;
    rc = upload_schedule(pb, hb, sp->bwd, std::max(sp->rmax64, sp->rmax32), fs.n, nnzL, fs.Lval);
    if (rc) return rc;
    CK(hipStreamSynchronize(pb->stream));
    fs.scheds.push_back(std::move(sp));
    SchedPair* last = fs.scheds.back().get();
    // the first strip whose slots fit: wider batches than its rmax are solved in column
    // chunks (fewer groups and crossings beat unchunked narrower strips)
    if ((fp32 ? last->rmax32 : last->rmax64) >= 1) {
      *out = last;
      return 0;
    }
  }
  return fail(pb, STOKES_EINVAL, "no triangular-solve schedule fits the LDS budget");
}

// Schedules of the IC(0) factor of A (any width: the solve kernel splits wide batches
// into column chunks).
int get_schedule(stokes_problem* pb, int R, bool fp32, SchedPair** out) {
  (void)R;
  return make_schedule(pb, pb->fsA, fp32, out);
}

int get_work(stokes_problem* pb, int R, bool fp32, Work** out) {
  const int key = R * 2 + (fp32 ? 1 : 0);
  auto it = pb->work.find(key);
  if (it != pb->work.end()) {
    *out = &it->second;
    return 0;
  }
  Work W;
  W.R = R;
  W.fp32 = fp32;
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  const size_t n = size_t(pb->S.n_u + pb->S.n_p) * R;
  const size_t nu = size_t(pb->S.n_u) * R;
  auto get = [&](size_t cnt) { return pb->mem.get<unsigned char>(cnt * es); };
  W.v[0] = get(n);
  W.v[1] = get(n);
  W.z[0] = get(n);
  W.z[1] = get(n);
  W.w[0] = get(n);
  W.w[1] = get(n);
  W.x = get(n);
  W.q = get(n);
  W.b = get(n);
  W.y = get(n);
  W.pr = get(nu);
  W.pp = get(nu);
  W.pq = get(nu);
  W.pz = get(nu);
  const size_t np = size_t(pb->S.n_p) * R;
  W.qr = get(np);
  W.qp = get(np);
  W.qq = get(np);
  W.qz = get(np);
  W.qy = get(np);
  if (pb->mem.err != hipSuccess) return fail_hip(pb, pb->mem.err, "workspace allocation", __LINE__);
  pb->work[key] = W;
  *out = &pb->work[key];
  return 0;
}

int check_trsv_err(stokes_problem* pb, const SchedPair* sp) {
  int e1 = 0, e2 = 0;
  CK(hipMemcpyAsync(&e1, sp->fwd.err, sizeof(int), hipMemcpyDeviceToHost, pb->stream));
  CK(hipMemcpyAsync(&e2, sp->bwd.err, sizeof(int), hipMemcpyDeviceToHost, pb->stream));
  CK(hipStreamSynchronize(pb->stream));
  if (e1 || e2) {
    hipMemsetAsync(sp->fwd.err, 0, sizeof(int), pb->stream);
    hipMemsetAsync(sp->bwd.err, 0, sizeof(int), pb->stream);
    hipStreamSynchronize(pb->stream);
    return fail(pb, STOKES_EHIP, "triangular solve: a device-side wait exceeded its spin limit");
  }
  return 0;
}

// Ideal(A,Q) (Sec. 5.1, exact block solves) is realised by Diag-preconditioned CG on A and
// on Q run to this relative residual, far below the outer tolerances the solver accepts,
// so that MINRES sees the fixed preconditioner blkdiag(A, Q/(2 nu)) up to rounding.
constexpr double kIdealTol = 1e-12;
// STOKES_MIXED refines the true residual to this fraction of the requested tolerance.
constexpr double kMixedMargin = 0.1;
constexpr int kIdealMaxit = 100000;

// Queue inner CG iterations (iter() queues one) until the device all-done flag is set or
// maxit are queued: a first chunk of 4 fewer than the previous application needed, then
// chunks of 4.  The flag written after chunk c is read while chunk c+1 is already queued,
// so the device does not wait for the host; at most one chunk runs after convergence, its
// launches returning at once.  *expect receives this application's largest count.
template <typename Iter>
int pcg_run(stokes_problem* pb, const PcgScalars& s, int R, int maxit, int* expect, Iter iter) {
  hipStream_t st = pb->stream;
  if (pb->pcg_hflag == nullptr) {
    CK(hipHostMalloc((void**)&pb->pcg_hflag, 2 * sizeof(int), hipHostMallocDefault));
    for (auto& e : pb->pcg_ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  int queued = 0, chunk = 0;
  bool done = false;
  while (queued < maxit && !done) {
    const int n = std::min(maxit - queued, chunk == 0 ? std::max(1, *expect - 4) : 4);
    for (int k = 0; k < n; ++k) CK(iter());
    queued += n;
    const int slot = chunk & 1;
    CK(hipMemcpyAsync(pb->pcg_hflag + slot, s.alldone, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipEventRecord(pb->pcg_ev[slot], st));
    if (chunk > 0) {
      CK(hipEventSynchronize(pb->pcg_ev[1 - slot]));
      done = pb->pcg_hflag[1 - slot] != 0;
      prof_flush(pb);
    }
    ++chunk;
  }
  PcgState ps[kRMax];
  CK(hipMemcpyAsync(ps, s.st, sizeof(PcgState) * R, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  int mx = 0;
  for (int c = 0; c < R; ++c) mx = std::max(mx, ps[c].iter);
  if (mx > 0) *expect = mx;
  prof_flush(pb);
  return 0;
}

// Velocity block of the preconditioner: zout_u = M_A^{-1} vin_u, and the dot v_u . z_u
// into dot_out[R].  skip: device flag (all columns done) or null.
template <typename T>
int precond_velocity(stokes_problem* pb, int precond, Work& W, SchedPair* sp, const T* vin, T* zout,
                     double* dot_out, const int* skip, const MinresState* outer_st, int* inner_total) {
  const int R = W.R;
  const bool fp32 = W.fp32;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u;
  if (precond == STOKES_PC_IC0) {
    CK(launch_trsv(sp->fwd, fp32, R, vin, W.y, nullptr, nullptr, skip, st, prof_take(pb, 1)));
    CK(launch_trsv(sp->bwd, fp32, R, W.y, zout, vin, dot_out, skip, st, prof_take(pb, 2)));
    return 0;
  }
  const bool ideal = precond == STOKES_PC_IDEAL || precond == STOKES_PC_IDEAL_A;
  const bool jacobi_cg = precond == STOKES_PC_JPCG || precond == STOKES_PC_PCGAQ || ideal;
  const bool ic_cg = precond == STOKES_PC_ICPCG || precond == STOKES_PC_ICPCG_AQ;
  if (ic_cg || jacobi_cg) {
    const double rtol_in = ideal ? kIdealTol : pb->inner_tol;
    const int maxit_in = ideal ? kIdealMaxit : pb->maxit_inner;
    int& expect = pb->pcg_expect[precond];
    const T* val = fp32 ? (const T*)pb->val32 : (const T*)pb->val;
    PcgScalars& s = pb->pcg;
    // z = M^{-1} r with rho = r.z: the IC(0) triangular solves (fused dot), or Jacobi
    auto inner_precond = [&](double* rho_out, const int* sk, bool prof) -> hipError_t {
      if (jacobi_cg)
        return pcg_jacobi<T>(R, n_u, (const T*)W.pr, pb->diagA, (T*)W.pz, s, rho_out, sk, st);
      hipError_t e = launch_trsv(sp->fwd, fp32, R, W.pr, W.y, nullptr, nullptr, sk, st, prof ? prof_take(pb, 1) : nullptr);
      if (e != hipSuccess) return e;
      return launch_trsv(sp->bwd, fp32, R, W.y, W.pz, W.pr, rho_out, sk, st, prof ? prof_take(pb, 2) : nullptr);
    };
    CK(pcg_init<T>(R, n_u, vin, (T*)W.pr, zout, s, skip, st));
    CK(inner_precond(s.rho, skip, false));
    CK(pcg_init2<T>(R, n_u, (const T*)W.pz, (T*)W.pp, s, rtol_in, maxit_in, skip, outer_st, st));
    int ip = 0;
    auto iter = [&]() -> hipError_t {
      hipError_t e = pcg_spmv<T>(R, pb->rs_A, pb->rowptr, pb->aend, pb->col, val, (const T*)W.pp, (T*)W.pq, s, ic_cg,
                                 st);
      if (e == hipSuccess && jacobi_cg)
        e = pcg_axpy_jacobi<T>(R, n_u, (const T*)W.pp, (const T*)W.pq, pb->diagA, zout, (T*)W.pr, (T*)W.pz, s, ip,
                               st);
      if (e == hipSuccess && !jacobi_cg) {
        e = pcg_axpy<T>(R, n_u, (const T*)W.pp, (const T*)W.pq, zout, (T*)W.pr, s, ip, st);
        if (e == hipSuccess) e = inner_precond(s.rho + (1 - ip) * kRMax, s.alldone, true);
      }
      if (e == hipSuccess) e = pcg_pupdate<T>(R, n_u, (const T*)W.pz, (T*)W.pp, s, ip, st);
      ip = 1 - ip;
      return e;
    };
    if (int e = pcg_run(pb, s, R, maxit_in, &expect, iter)) return e;
    CK(dot<T, T>(R, 0, n_u, vin, zout, pb->partials, pb->counter, dot_out, st));
    (void)inner_total;
    return 0;
  }
  return 0;  // Jacobi: handled inside the vector kernels
}

// Q in CSR (pattern of overlapping pressure supports, values by quadrature) and the
// pressure-block CG scalars, built on first use.
int ensure_pressure_cg(stokes_problem* pb) {
  if (pb->Qval != nullptr) return 0;
  const Spaces& S = pb->S;
  const int nlo = S.nlo, kp = S.kp, dim = S.dim;
  const int64_t np = S.n_p;
  std::vector<int32_t>& rp = pb->Qrowptr_h;
  std::vector<int32_t>& cl = pb->Qcol_h;
  cl.clear();
  rp.assign(size_t(np) + 1, 0);
  for (int64_t r = 0; r < np; ++r) {
    int i[3] = {int(r % nlo), dim > 1 ? int((r / nlo) % nlo) : 0, dim > 2 ? int(r / (int64_t(nlo) * nlo)) : 0};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = d < dim ? std::max(0, i[d] - kp) : 0;
      hi[d] = d < dim ? std::min(nlo - 1, i[d] + kp) : 0;
    }
    for (int j2 = lo[2]; j2 <= hi[2]; ++j2)
      for (int j1 = lo[1]; j1 <= hi[1]; ++j1)
        for (int j0 = lo[0]; j0 <= hi[0]; ++j0) cl.push_back(int32_t(j0 + int64_t(nlo) * (j1 + int64_t(nlo) * j2)));
    rp[size_t(r) + 1] = int32_t(cl.size());
  }
  DevAlloc& m = pb->mem;
  hipStream_t st = pb->stream;
  pb->Qrowptr = m.upload(rp, st);
  pb->Qcol = m.upload(cl, st);
  pb->Qval = m.get<double>(cl.size());
  pb->Qval32 = m.get<float>(cl.size());
  pb->rs_Q.nb = row_split_blocks(np, pb->num_cu, kPcgSpmvBlocksPerCU);
  pb->split_Q_h = balanced_row_split(rp, nullptr, np, pb->rs_Q.nb);
  pb->rs_Q.split = m.upload(pb->split_Q_h, st);
  pb->pcgQ.st = m.get<PcgState>(kRMax);
  pb->pcgQ.alldone = m.get<int>(1);
  pb->pcgQ.rho = m.get<double>(2 * kRMax);
  pb->pcgQ.pq = m.get<double>(kRMax);
  pb->pcgQ.rr = m.get<double>(kRMax);
  pb->pcgQ.partials = pb->partials;
  pb->pcgQ.counter = pb->counter + 2;
  if (m.err != hipSuccess) return fail_hip(pb, m.err, "pressure-block CG allocation", __LINE__);
  CK(hipMemsetAsync(pb->pcgQ.st, 0, kRMax * sizeof(PcgState), st));
  CK(assemble_Q(S, pb->Qrowptr, pb->Qcol, pb->Qval, st));
  CK(convert<double, float>(int64_t(cl.size()), pb->Qval, pb->Qval32, st));
  CK(hipStreamSynchronize(st));  // the host vectors must outlive the copies
  return 0;
}

// IC(0) of the pressure mass matrix Q on the pattern of tril(Q) in natural order, and its
// triangular-solve schedules (pressure rows in strips of the last direction), built on
// first use.  Q is SPD; a non-positive pivot is reported as a breakdown (no shifts).
int ensure_pressure_ic0(stokes_problem* pb) {
  if (pb->LQval != nullptr) return 0;
  int rc = ensure_pressure_cg(pb);
  if (rc) return rc;
  const Spaces& S = pb->S;
  const int64_t np = S.n_p;
  LowerPattern& L = pb->LQ;
  L.rowptr.assign(size_t(np) + 1, 0);
  L.col.clear();
  L.src.clear();
  for (int64_t r = 0; r < np; ++r) {  // Q's columns are sorted: the diagonal ends the lower part
    for (int32_t k = pb->Qrowptr_h[r]; k < pb->Qrowptr_h[r + 1]; ++k) {
      if (pb->Qcol_h[k] > r) break;
      L.col.push_back(pb->Qcol_h[k]);
      L.src.push_back(k);
    }
    if (L.col.empty() || L.col.back() != r) return fail(pb, STOKES_EINVAL, "pressure mass matrix without a diagonal");
    L.rowptr[size_t(r) + 1] = int32_t(L.col.size());
  }
  int nlev = 0;
  forward_levels(L, np, pb->levQ_fwd, &nlev);
  std::vector<int32_t> lptr(size_t(nlev) + 1, 0), rows(static_cast<size_t>(np));
  for (int64_t i = 0; i < np; ++i) lptr[pb->levQ_fwd[i] + 1]++;
  for (int l = 0; l < nlev; ++l) lptr[l + 1] += lptr[l];
  std::vector<int32_t> fillp(lptr.begin(), lptr.end() - 1);
  for (int64_t i = 0; i < np; ++i) rows[fillp[pb->levQ_fwd[i]]++] = int32_t(i);
  DevAlloc& m = pb->mem;
  hipStream_t st = pb->stream;
  pb->LQrowptr = m.upload(L.rowptr, st);
  pb->LQcol = m.upload(L.col, st);
  pb->LQsrc = m.upload(L.src, st);
  int32_t* lrows = m.upload(rows, st);
  double* lqval = m.get<double>(L.col.size());
  if (m.err != hipSuccess) return fail_hip(pb, m.err, "IC(0) of Q allocation", __LINE__);
  CK(ic0_factor(np, int64_t(L.col.size()), pb->LQsrc, pb->LQrowptr, pb->LQcol, pb->Qval, 0.0, lqval, lrows, lptr,
                pb->flag, st));
  int fl = 0;
  CK(hipMemcpyAsync(&fl, pb->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));  // also: the host vectors outlive the copies
  if (fl >= 0) return fail(pb, STOKES_EBREAKDOWN, "IC(0) of the pressure mass matrix: non-positive pivot");
  FactorSched& fs = pb->fsQ;
  fs.L = &pb->LQ;
  fs.n = np;
  fs.Lval = lqval;
  fs.lev_fwd = &pb->levQ_fwd;
  fs.lev_bwd = &pb->levQ_bwd;
  fs.groups = [pb](int strip, std::vector<int32_t>& g, int* ng) {
    // pressure row r has last-direction index r / inner
    const Spaces& S = pb->S;
    int64_t inner = 1;
    for (int d = 0; d + 1 < S.dim; ++d) inner *= S.nlo;
    g.assign(size_t(S.n_p), 0);
    for (int64_t r = 0; r < S.n_p; ++r) g[size_t(r)] = int32_t((r / inner) / strip);
    *ng = int((S.nlo + strip - 1) / strip);
  };
  SchedPair* sp = nullptr;
  rc = make_schedule(pb, fs, false, &sp);
  if (rc) return rc;
  pb->LQval = lqval;
  return 0;
}

// Pressure block of the PCG(A,Q) and Ideal(A,Q) preconditioners: zout_p = 2 nu Q^{-1} vin_p
// by Diag(Q)-preconditioned CG (x0 = 0, relative tolerance inner_tol, or kIdealTol for
// Ideal(A,Q)), and the dot v_p . z_p into dot_out[R].  vin_p / zout_p point at the pressure
// rows (row n_u).
// Inner solver of the pressure block.
enum { PQ_CG_JACOBI = 0, PQ_CG_IDEAL = 1, PQ_CG_IC0 = 2 };

template <typename T>
int precond_pressure(stokes_problem* pb, Work& W, int kind, const T* vin_p, T* zout_p, double* dot_out,
                     const int* skip, const MinresState* outer_st, double rtol_set = 0.0, int maxit_set = 0) {
  const int R = W.R;
  const bool fp32 = W.fp32;
  hipStream_t st = pb->stream;
  const int64_t n_p = pb->S.n_p;
  const T* qval = fp32 ? (const T*)pb->Qval32 : (const T*)pb->Qval;
  PcgScalars& s = pb->pcgQ;
  const bool ic0 = kind == PQ_CG_IC0;
  SchedPair* qsp = nullptr;
  if (ic0) {
    int rc = ensure_pressure_ic0(pb);
    if (rc) return rc;
    if ((rc = make_schedule(pb, pb->fsQ, fp32, &qsp))) return rc;
  }
  // z = M^{-1} r with rho = r.z: Jacobi, or the IC(0) triangular solves of Q (fused dot)
  auto inner_precond = [&](double* rho_out, const int* sk) -> hipError_t {
    if (!ic0) return pcg_jacobi<T>(R, n_p, (const T*)W.qr, pb->diagQ, (T*)W.qz, s, rho_out, sk, st);
    hipError_t e = launch_trsv(qsp->fwd, fp32, R, W.qr, W.qy, nullptr, nullptr, sk, st);
    if (e != hipSuccess) return e;
    return launch_trsv(qsp->bwd, fp32, R, W.qy, W.qz, W.qr, rho_out, sk, st);
  };
  CK(pcg_init<T>(R, n_p, vin_p, (T*)W.qr, zout_p, s, skip, st));
  CK(inner_precond(s.rho, skip));
  const double rtol_in = rtol_set > 0.0 ? rtol_set : (kind == PQ_CG_IDEAL ? kIdealTol : pb->inner_tol);
  const int maxit_in = maxit_set > 0 ? maxit_set : (kind == PQ_CG_IDEAL ? kIdealMaxit : pb->maxit_inner);
  int& expect = pb->pcgq_expect[kind];
  CK(pcg_init2<T>(R, n_p, (const T*)W.qz, (T*)W.qp, s, rtol_in, maxit_in, skip, outer_st, st));
  int ip = 0;
  auto iter = [&]() -> hipError_t {
    hipError_t e = pcg_spmv<T>(R, pb->rs_Q, pb->Qrowptr, nullptr, pb->Qcol, qval, (const T*)W.qp, (T*)W.qq, s, false, st);
    if (e == hipSuccess && !ic0)
      e = pcg_axpy_jacobi<T>(R, n_p, (const T*)W.qp, (const T*)W.qq, pb->diagQ, zout_p, (T*)W.qr, (T*)W.qz, s, ip, st);
    if (e == hipSuccess && ic0) {
      e = pcg_axpy<T>(R, n_p, (const T*)W.qp, (const T*)W.qq, zout_p, (T*)W.qr, s, ip, st);
      if (e == hipSuccess) e = inner_precond(s.rho + (1 - ip) * kRMax, s.alldone);
    }
    if (e == hipSuccess) e = pcg_pupdate<T>(R, n_p, (const T*)W.qz, (T*)W.qp, s, ip, st);
    ip = 1 - ip;
    return e;
  };
  if (int e = pcg_run(pb, s, R, maxit_in, &expect, iter)) return e;
  if (qsp) {
    int rc = check_trsv_err(pb, qsp);
    if (rc) return rc;
  }
  CK(scale_skip<T>(n_p * R, zout_p, 2.0 * pb->nu, skip, st));
  CK(dot<T, T>(R, 0, n_p, vin_p, zout_p, pb->partials, pb->counter, dot_out, st));
  return 0;
}

// Pressure-block inner solver of a preconditioner code (-1: Diag(Q) in the vector kernels).
int pressure_kind(int precond) {
  if (precond == STOKES_PC_PCGAQ) return PQ_CG_JACOBI;
  if (precond == STOKES_PC_IDEAL) return PQ_CG_IDEAL;
  if (precond == STOKES_PC_ICPCG_AQ) return PQ_CG_IC0;
  return -1;
}

struct RunOut {
  int iters[kRMax];
  int status[kRMax];
  double eta[kRMax], gamma1[kRMax];
};

// MINRES on Acal x = b (b in W.b, x out in W.x), R columns, precision of W.
template <typename T>
int minres_run(stokes_problem* pb, Work& W, int precond, double tol, int maxit, RunOut& ro) {
  const int R = W.R;
  const bool fp32 = W.fp32;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n = n_u + pb->S.n_p;
  SchedPair* sp = nullptr;
  if (precond == STOKES_PC_IC0 || precond == STOKES_PC_ICPCG || precond == STOKES_PC_ICPCG_AQ) {
    int rc = get_schedule(pb, R, fp32, &sp);
    if (rc) return rc;
  }
  const int qkind = pressure_kind(precond);
  const bool pcg_q = qkind >= 0;
  if (pcg_q) {
    int rc = ensure_pressure_cg(pb);
    if (rc) return rc;
  }
  const T* val = fp32 ? (const T*)pb->val32 : (const T*)pb->val;
  const double* diagA = precond == STOKES_PC_JACOBI ? pb->diagA : nullptr;
  const double two_nu = 2.0 * pb->nu;
  MrScalars& s = pb->mr;
  T* v[2] = {(T*)W.v[0], (T*)W.v[1]};
  T* z[2] = {(T*)W.z[0], (T*)W.z[1]};
  T* w[2] = {(T*)W.w[0], (T*)W.w[1]};
  T* x = (T*)W.x;
  T* q = (T*)W.q;
  CK(mr_init_vec<T>(R, n, n_u, (const T*)W.b, v[0], v[1], w[0], w[1], x, z[0], pb->diagQ, diagA, two_nu, s, st));
  // the outer state is not initialised yet: no outer-done test for this application
  int rc = precond_velocity<T>(pb, precond, W, sp, v[0], z[0], s.red + RED_G2U * kRMax, nullptr, nullptr, nullptr);
  if (rc) return rc;
  if (pcg_q) {  // the pressure block replaces the Diag(Q) part the vector kernel wrote
    rc = precond_pressure<T>(pb, W, qkind, v[0] + n_u * R, z[0] + n_u * R, s.red + RED_G2P * kRMax, nullptr, nullptr);
    if (rc) return rc;
  }
  CK(mr_init_state(R, s, tol, maxit, st));
  if (pb->hflag == nullptr) {
    CK(hipHostMalloc((void**)&pb->hflag, 2 * sizeof(int), hipHostMallocDefault));
    for (auto& e : pb->flag_ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // Iterations are enqueued in chunks of check_every.  After enqueueing chunk k the host
  // waits for the done flag of chunk k-1 only, so the device always has a chunk queued;
  // iterations after convergence return at once (device-side done flags).
  int j = 1, chunk = 0;
  for (;;) {
    for (int m = 0; m < pb->check_every; ++m, ++j) {
      const int p = (j - 1) & 1;
      {
        PROF_BEGIN(0);
        CK(mr_spmv<T>(R, pb->rs_full, pb->rowptr, pb->col, val, z[p], q, s, p, pb->spmv_nt, st));
        PROF_END();
      }
      {
        PROF_BEGIN(3);
        CK(mr_lanczos<T>(R, n, n_u, q, v[p], v[1 - p], z[1 - p], pb->diagQ, diagA, two_nu, s, p, st));
        PROF_END();
      }
      rc = precond_velocity<T>(pb, precond, W, sp, v[1 - p], z[1 - p],
                               s.red + ((size_t)p * RED_KINDS + RED_G2U) * kRMax, s.alldone + p, s.st + p * kRMax,
                               nullptr);
      if (rc) return rc;
      if (pcg_q) {
        rc = precond_pressure<T>(pb, W, qkind, v[1 - p] + n_u * R, z[1 - p] + n_u * R,
                                 s.red + ((size_t)p * RED_KINDS + RED_G2P) * kRMax, s.alldone + p, s.st + p * kRMax);
        if (rc) return rc;
      }
      {
        PROF_BEGIN(4);
        CK(mr_update<T>(R, n, z[p], w[p], w[1 - p], x, s, p, st));
        PROF_END();
      }
    }
    const int slot = chunk & 1;
    CK(hipMemcpyAsync(pb->hflag + slot, s.alldone + ((j - 1) & 1), sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipEventRecord(pb->flag_ev[slot], st));
    const bool over = j > maxit + 2 * pb->check_every + 1;
    if (chunk > 0 || over) {
      const int ws = over ? slot : 1 - slot;
      CK(hipEventSynchronize(pb->flag_ev[ws]));
      prof_flush(pb);
      if (pb->hflag[ws] || over) break;
    }
    ++chunk;
  }
  CK(hipStreamSynchronize(st));
  prof_flush(pb);
  const int fp = (j - 1) & 1;
  MinresState hs[kRMax];
  CK(hipMemcpyAsync(hs, s.st + fp * kRMax, sizeof(MinresState) * kRMax, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (int c = 0; c < R; ++c) {
    ro.iters[c] = hs[c].iter;
    ro.status[c] = hs[c].status;
    ro.eta[c] = hs[c].eta;
    ro.gamma1[c] = hs[c].gamma1;
  }
  if (sp) {
    rc = check_trsv_err(pb, sp);
    if (rc) return rc;
  }
  return 0;
}

// Zero-mean pressure of the interleaved double vector x (R columns).
int project_pressure(stokes_problem* pb, int R, double* x) {
  const int64_t n_u = pb->S.n_u, n_p = pb->S.n_p;
  R_SWITCH(R, hipLaunchKernelGGL((k_pdot<RR>), dim3(vec_blocks(n_p)), dim3(kVT), 0, pb->stream, n_p, n_u, pb->w, x,
                                 pb->partials, pb->counter, pb->scratch));
  CK(hipGetLastError());
  CK(sub_mean<double>(R, n_u, n_u + n_p, x, pb->scratch, pb->w1, pb->kappa, pb->stream));
  return 0;
}

// True residual norms of the interleaved double solution x for right-hand side b:
// rel2[c] = ||b - Acal x||_2/||b||_2 and relM[c] = ||r||_{M^-1}/||b||_{M^-1} (IC(0) or
// Jacobi M).  Uses work buffers of the FP64 workspace W (q, y, and v[0] as scratch).
int true_residuals(stokes_problem* pb, Work& W, int precond, const double* b, const double* x, double* rel2,
                   double* relM) {
  const int R = W.R;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n = n_u + pb->S.n_p;
  double* r = (double*)W.q;
  double* out = pb->scratch;  // [0..2R) norms, [2R..4R) r M r parts, [4R..6R) b M b parts
  CK(spmv_resid<double>(R, pb->rs_full, pb->rowptr, nullptr, pb->col, pb->val, x, b, r, pb->partials, pb->counter, out, st));
  const int pcl = (precond == STOKES_PC_JACOBI || precond == STOKES_PC_JPCG || precond == STOKES_PC_PCGAQ ||
                   precond == STOKES_PC_IDEAL || precond == STOKES_PC_IDEAL_A)
                      ? STOKES_PC_JACOBI
                      : STOKES_PC_IC0;
  // IC(0)-PCG on Q approximates the fixed pressure block IC(0) of Q / (2 nu)
  const bool icq = precond == STOKES_PC_ICPCG_AQ;
  if (icq) {
    int rc = ensure_pressure_ic0(pb);
    if (rc) return rc;
  }
  for (int pass = 0; pass < 2; ++pass) {
    const double* vec = pass == 0 ? r : b;
    double* o = out + 2 * R + pass * 2 * R;
    R_SWITCH(R, hipLaunchKernelGGL((k_diag_wsq<RR>), dim3(vec_blocks(n)), dim3(kVT), 0, st, n_u, n, vec, pb->diagQ,
                                   pcl == STOKES_PC_JACOBI ? pb->diagA : nullptr, 2.0 * pb->nu, pb->partials,
                                   pb->counter, o));
    CK(hipGetLastError());
    if (pcl == STOKES_PC_IC0) {
      SchedPair* sp = nullptr;
      int rc = get_schedule(pb, R, false, &sp);
      if (rc) return rc;
      CK(launch_trsv(sp->fwd, false, R, vec, W.y, nullptr, nullptr, nullptr, st));
      CK(launch_trsv(sp->bwd, false, R, W.y, W.v[0], vec, o + R, nullptr, st));
    }
    if (icq) {  // pressure part r_p . (L_Q L_Q^T)^{-1} r_p, scaled by 2 nu below
      SchedPair* qsp = nullptr;
      int rc = make_schedule(pb, pb->fsQ, false, &qsp);
      if (rc) return rc;
      const double* vp = vec + size_t(n_u) * R;
      CK(launch_trsv(qsp->fwd, false, R, vp, W.qy, nullptr, nullptr, nullptr, st));
      CK(launch_trsv(qsp->bwd, false, R, W.qy, W.qz, vp, o, nullptr, st));
    }
  }
  double h[6 * kRMax];
  CK(hipMemcpyAsync(h, out, sizeof(double) * 6 * R, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  const double sp_ = icq ? 2.0 * pb->nu : 1.0;
  for (int c = 0; c < R; ++c) {
    const double rr = h[c], bb = h[R + c];
    const double rM = sp_ * h[2 * R + c] + h[3 * R + c], bM = sp_ * h[4 * R + c] + h[5 * R + c];
    rel2[c] = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    relM[c] = bM > 0 ? std::sqrt(std::max(0.0, rM) / bM) : 0.0;
  }
  return 0;
}

int validate_vec(stokes_problem* pb, const void* p, const char* name) {
  if (p == nullptr) return fail(pb, STOKES_EINVAL, std::string("null pointer: ") + name);
  return 0;
}

int round_r(int nrhs) { return nrhs <= 1 ? 1 : (nrhs <= 8 ? 8 : 16); }

// Common driver: RHS already in the FP64 workspace W64.b (interleaved, R columns).
// Solves in the requested precision; the solution lands in W64.x (FP64, projected).
int solve_core(stokes_problem* pb, Work& W64, int precond, int precision, double tol, stokes_info* infos, int nrhs) {
  const int R = W64.R;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n = n_u + pb->S.n_p;
  RunOut ro;
  int iters_total[kRMax] = {0};
  int status[kRMax] = {0};
  double eta_rel[kRMax] = {0};
  int cycles = 1;
  const bool inner_pcg = precond == STOKES_PC_ICPCG || precond == STOKES_PC_JPCG || precond == STOKES_PC_PCGAQ ||
                         precond == STOKES_PC_ICPCG_AQ;
  // Ideal(A,Q), Ideal(A) + Diag(Q): fixed preconditioners up to rounding, one MINRES run
  // (no restarts)
  const bool pcg_q = pressure_kind(precond) >= 0;
  const bool counts_inner = inner_pcg || precond == STOKES_PC_IDEAL || precond == STOKES_PC_IDEAL_A;
  // inner CG totals count over every refinement cycle of this solve
  if (counts_inner) {
    CK(hipMemsetAsync(pb->pcg.st, 0, sizeof(PcgState) * kRMax, st));
    if (pcg_q) {
      int rc = ensure_pressure_cg(pb);
      if (rc) return rc;
      CK(hipMemsetAsync(pb->pcgQ.st, 0, sizeof(PcgState) * kRMax, st));
    }
  }
  // inner CG to a relative tolerance: one MINRES run as in Sec. 5.1 unless restarts on the
  // true residual were asked for (stokes_set_restarts)
  const bool restarted = inner_pcg && pb->restarts > 0;
  if (precision == STOKES_FP64 && !restarted) {
    int rc = minres_run<double>(pb, W64, precond, tol, pb->maxit_outer, ro);
    if (rc) return rc;
    for (int c = 0; c < R; ++c) {
      iters_total[c] = ro.iters[c];
      status[c] = ro.status[c];
      eta_rel[c] = ro.gamma1[c] > 0 ? std::fabs(ro.eta[c]) / ro.gamma1[c] : 0.0;
    }
    int rc2 = project_pressure(pb, R, (double*)W64.x);
    if (rc2) return rc2;
  } else if (precision == STOKES_FP64) {
    // Inner CG to a relative tolerance is a nonlinear preconditioner: MINRES's |eta| then
    // measures the residual in a norm that changes from one application to the next.
    // Refine on the true residual (FP64, M = IC(0) or Diag(A) on the velocity block) until
    // it meets the tolerance.
    if (W64.xr == nullptr) {
      W64.xr = pb->mem.get<double>(size_t(n) * R);
      W64.br = pb->mem.get<double>(size_t(n) * R);
      if (pb->mem.err != hipSuccess) return fail_hip(pb, pb->mem.err, "refinement workspace", __LINE__);
      for (auto& kv : pb->work)
        if (kv.second.R == R && !kv.second.fp32) {
          kv.second.xr = W64.xr;
          kv.second.br = W64.br;
        }
    }
    double* xacc = (double*)W64.xr;
    double* b0 = (double*)W64.br;
    double* b = (double*)W64.b;
    hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, st, int64_t(n * R), xacc, 0.0);
    CK(hipMemcpyAsync(b0, b, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
    double rel2[kRMax], relM[kRMax];
    double tol_k = tol;
    bool conv = false;
    cycles = 0;
    for (int ir = 0; ir < pb->restarts && !conv; ++ir) {
      int rc = minres_run<double>(pb, W64, precond, tol_k, pb->maxit_outer, ro);
      if (rc) return rc;
      ++cycles;
      for (int c = 0; c < R; ++c) {
        iters_total[c] += ro.iters[c];
        if (ro.status[c] < 0) status[c] = ro.status[c];
      }
      CK(accumulate<double>(R, int64_t(n * R), xacc, (const double*)W64.x, st));
      rc = project_pressure(pb, R, xacc);
      if (rc) return rc;
      rc = true_residuals(pb, W64, precond, b0, xacc, rel2, relM);
      if (rc) return rc;
      double worst = 0.0;
      conv = true;
      for (int c = 0; c < R; ++c) {
        conv &= (relM[c] <= tol);
        worst = std::max(worst, relM[c]);
      }
      // next cycle solves Acal d = r (r left in W64.q) to the remaining relative reduction
      CK(hipMemcpyAsync(b, W64.q, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
      tol_k = worst > 0.0 ? std::min(0.5, 0.5 * tol / worst) : tol;
    }
    CK(hipMemcpyAsync(W64.x, xacc, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(b, b0, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
    for (int c = 0; c < R; ++c) {
      if (status[c] >= 0) status[c] = relM[c] <= tol ? 0 : STOKES_NOT_CONVERGED;
      eta_rel[c] = relM[c];
    }
  } else {
    // Iterative refinement: FP64 residual, FP32 inner MINRES, FP64 accumulation.
    Work* W32 = nullptr;
    int rc = get_work(pb, R, true, &W32);
    if (rc) return rc;
    double* x64 = (double*)W64.x;
    double* r64 = (double*)W64.z[1];
    double* b64 = (double*)W64.b;
    hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, st, int64_t(n * R), x64, 0.0);
    CK(hipMemcpyAsync(r64, b64, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
    double rel2[kRMax], relM[kRMax];
    for (int c = 0; c < kRMax; ++c) rel2[c] = relM[c] = HUGE_VAL;
    bool conv = false;
    // The refinement runs to tol * kMixedMargin: the error of an iterate is about
    // cond * residual, and at the margin the mixed solution stays within the FP64 solution's
    // error bar (measured at N = 512, k' = 2: 1.8e-8 relative error in u at a true residual
    // of 5e-9).  The first cycle asks the FP32 MINRES for refine_tol; later ones only for the
    // reduction that remains (with a factor 2 of margin), never more than refine_tol per cycle.
    const double target = tol * kMixedMargin;
    double tol_k = pb->refine_tol;
    cycles = 0;
    for (int ir = 0; ir < 30 && !conv; ++ir) {
      CK(convert<double, float>(int64_t(n * R), r64, (float*)W32->b, st));
      rc = minres_run<float>(pb, *W32, precond, tol_k, pb->maxit_outer, ro);
      if (rc) return rc;
      ++cycles;
      for (int c = 0; c < R; ++c) {
        iters_total[c] += ro.iters[c];
        if (ro.status[c] < 0) status[c] = ro.status[c];  // a breakdown of any cycle is kept
      }
      bool broke = false;
      for (int c = 0; c < R; ++c) broke |= status[c] < 0;
      if (broke) break;
      CK(accumulate<float>(R, int64_t(n * R), x64, (const float*)W32->x, st));
      rc = project_pressure(pb, R, x64);
      if (rc) return rc;
      rc = true_residuals(pb, W64, precond, b64, x64, rel2, relM);
      if (rc) return rc;
      // refresh r64 = b - Acal x (true_residuals left it in W64.q)
      CK(hipMemcpyAsync(r64, W64.q, sizeof(double) * n * R, hipMemcpyDeviceToDevice, st));
      conv = true;
      double worst = 0.0;
      for (int c = 0; c < R; ++c) {
        conv &= (relM[c] <= target);
        worst = std::max(worst, relM[c]);
      }
      tol_k = worst > 0.0 ? std::min(0.5, std::max(pb->refine_tol, 0.5 * target / worst)) : pb->refine_tol;
    }
    for (int c = 0; c < R; ++c) {
      if (status[c] >= 0) status[c] = relM[c] <= tol ? 0 : STOKES_NOT_CONVERGED;
      eta_rel[c] = relM[c];
    }
  }
  if (infos) {
    double rel2[kRMax], relM[kRMax];
    int rc = true_residuals(pb, W64, precond, (const double*)W64.b, (const double*)W64.x, rel2, relM);
    if (rc) return rc;
    for (int c = 0; c < nrhs; ++c) {
      infos[c].iters = iters_total[c];
      infos[c].status = status[c];
      infos[c].ic_shift_steps = pb->ic_shift_steps;
      infos[c].relres_est = eta_rel[c];
      infos[c].relres_true_2 = rel2[c];
      infos[c].relres_true_Minv = relM[c];
      infos[c].setup_ms = pb->setup_ms;
      infos[c].inner_iters_total = 0;
      infos[c].refine_cycles = cycles;
      infos[c].reserved = 0;
    }
    if (counts_inner) {
      PcgState ps[kRMax], pq[kRMax];
      CK(hipMemcpyAsync(ps, pb->pcg.st, sizeof(PcgState) * kRMax, hipMemcpyDeviceToHost, st));
      if (pcg_q) CK(hipMemcpyAsync(pq, pb->pcgQ.st, sizeof(PcgState) * kRMax, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      for (int c = 0; c < nrhs; ++c) infos[c].inner_iters_total = ps[c].total + (pcg_q ? pq[c].total : 0);
    }
  }
  int worst = 0;
  for (int c = 0; c < nrhs; ++c) {
    if (status[c] < 0) return fail(pb, status[c], "MINRES breakdown (negative gamma^2)");
    if (status[c] > 0) worst = STOKES_NOT_CONVERGED;
  }
  if (worst) pb->err = "MINRES did not reach the tolerance within the iteration limit";
  return worst;
}

int check_args_solve(stokes_problem* pb, double tol, int precond, int precision) {
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(pb, STOKES_EINVAL, "tol must be in (0, 1)");
  if (precond < 0 || precond > 7) return fail(pb, STOKES_EINVAL, "unknown preconditioner");
  if (precision != STOKES_FP64 && precision != STOKES_MIXED) return fail(pb, STOKES_EINVAL, "unknown precision");
  if ((precond == STOKES_PC_IDEAL || precond == STOKES_PC_IDEAL_A) && precision != STOKES_FP64)
    return fail(pb, STOKES_EINVAL, "the Ideal preconditioners need STOKES_FP64 (their inner tolerance is below FP32 rounding)");
  return 0;
}

// NaN/Inf check of a device input through a reduction of squares.
int check_finite(stokes_problem* pb, int R, const double* interleaved, int64_t len) {
  CK(dot<double, double>(1, 0, len * R, interleaved, interleaved, pb->partials, pb->counter, pb->scratch + 60,
                         pb->stream));
  double s = 0.0;
  CK(hipMemcpyAsync(&s, pb->scratch + 60, sizeof(double), hipMemcpyDeviceToHost, pb->stream));
  CK(hipStreamSynchronize(pb->stream));
  if (!std::isfinite(s)) return fail(pb, STOKES_EINVAL, "input contains NaN or Inf");
  return 0;
}

}  // namespace

// ===========================================================================
// extern "C" entry points
// ===========================================================================
extern "C" {

static int stokes_setup_impl(int n, int p, int dim, double nu, int geometry, double c_pen, stokes_problem* pb);

int stokes_setup(int n, int p, int dim, double nu, stokes_problem** out) {
  return stokes_setup_nitsche(n, p, dim, nu, STOKES_GEOMETRY_SQUARE, -1.0, out);
}

int stokes_setup_geometry(int n, int p, int dim, double nu, int geometry, stokes_problem** out) {
  return stokes_setup_nitsche(n, p, dim, nu, geometry, -1.0, out);
}

int stokes_setup_nitsche(int n, int p, int dim, double nu, int geometry, double c_pen, stokes_problem** out) {
  if (out == nullptr) return STOKES_EINVAL;
  *out = nullptr;
  if (n < 1 || n > 4096 || p < 1 || p > 3 || (dim != 2 && dim != 3) || !(nu > 0.0) || !std::isfinite(nu))
    return STOKES_EINVAL;
  if (geometry != STOKES_GEOMETRY_SQUARE && !(geometry == STOKES_GEOMETRY_ANNULUS && dim == 2)) return STOKES_EINVAL;
  if (!std::isfinite(c_pen)) return STOKES_EINVAL;
  stokes_problem* pb = new stokes_problem();
  const int rc = stokes_setup_impl(n, p, dim, nu, geometry, c_pen, pb);
  if (rc != 0) {
    if (!pb->err.empty()) fprintf(stderr, "stokes_setup: %s\n", pb->err.c_str());
    (void)hipStreamSynchronize(pb->stream);
    delete pb;
    return rc;
  }
  *out = pb;
  return 0;
}

static int stokes_setup_impl(int n, int p, int dim, double nu, int geometry, double c_pen, stokes_problem* pb) {
  auto t0 = std::chrono::steady_clock::now();
  pb->S = make_spaces(n, p, dim);
  pb->S.geom = geometry;
  pb->nu = nu;
  pb->cpen = c_pen < 0.0 ? 5.0 * (p + 1) : c_pen;
  int dev = 0;
  CK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, dev));
  pb->lds_max = prop.sharedMemPerBlock;
  pb->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor > 0 ? prop.maxSharedMemoryPerMultiProcessor
                                                              : prop.sharedMemPerBlock;
  pb->num_cu = prop.multiProcessorCount;
  std::string e;
  if (build_saddle_pattern(pb->S, pb->P, e) != 0) return fail(pb, STOKES_EINVAL, e);
  build_lower_pattern(pb->S, pb->P, pb->L);
  {
    int maxrow = 0;
    for (int64_t i = 0; i < pb->S.n_u; ++i) maxrow = std::max(maxrow, pb->L.rowptr[i + 1] - pb->L.rowptr[i]);
    if (maxrow > 128) return fail(pb, STOKES_EINVAL, "IC(0) rows longer than 128 entries are not supported");
  }
  const int64_t nall = pb->S.n_u + pb->S.n_p;
  pb->nnz = int64_t(pb->P.col.size());
  pb->nnzL = int64_t(pb->L.col.size());
  hipStream_t st = pb->stream;
  DevAlloc& m = pb->mem;
  pb->rowptr = m.upload(pb->P.rowptr, st);
  pb->col = m.upload(pb->P.col, st);
  pb->aend = m.upload(pb->P.aend, st);
  {
    const int64_t n_all = pb->S.n_u + pb->S.n_p;
    const int nbf = row_split_blocks(n_all, pb->num_cu);
    const int nba = row_split_blocks(pb->S.n_u, pb->num_cu, kPcgSpmvBlocksPerCU);
    pb->split_full_h = balanced_row_split(pb->P.rowptr, nullptr, n_all, nbf);
    pb->split_A_h = balanced_row_split(pb->P.rowptr, &pb->P.aend, pb->S.n_u, nba);
    pb->rs_full.nb = nbf;
    pb->rs_full.split = m.upload(pb->split_full_h, st);
    pb->rs_A.nb = nba;
    pb->rs_A.split = m.upload(pb->split_A_h, st);
  }
  pb->val = m.get<double>(pb->nnz);
  pb->val32 = m.get<float>(pb->nnz);
  pb->diagQ = m.get<double>(pb->S.n_p);
  pb->w = m.get<double>(pb->S.n_p);
  pb->diagA = m.get<double>(pb->S.n_u);
  pb->Lrowptr = m.upload(pb->L.rowptr, st);
  pb->Lcol = m.upload(pb->L.col, st);
  pb->Lsrc = m.upload(pb->L.src, st);
  pb->Lval = m.get<double>(pb->nnzL);
  pb->flag = m.get<int>(4);
  pb->scratch = m.get<double>(128);
  pb->partials = m.get<double>(size_t(kVecMaxBlocks) * 2 * kRMax + 64);
  pb->counter = m.get<unsigned int>(16);
  pb->mr.st = m.get<MinresState>(2 * kRMax);
  pb->mr.alldone = m.get<int>(2);
  pb->mr.red = m.get<double>(2 * RED_KINDS * kRMax);
  pb->mr.partials = pb->partials;
  pb->mr.counter = pb->counter;
  pb->pcg.st = m.get<PcgState>(kRMax);
  pb->pcg.alldone = m.get<int>(1);
  pb->pcg.rho = m.get<double>(2 * kRMax);
  pb->pcg.pq = m.get<double>(kRMax);
  pb->pcg.rr = m.get<double>(kRMax);
  pb->pcg.partials = pb->partials;
  pb->pcg.counter = pb->counter + 1;
  if (m.err != hipSuccess) return fail_hip(pb, m.err, "allocation", __LINE__);
  CK(hipMemsetAsync(pb->counter, 0, 16 * sizeof(unsigned int), st));
  CK(hipMemsetAsync(pb->mr.red, 0, 2 * RED_KINDS * kRMax * sizeof(double), st));
  CK(hipMemsetAsync(pb->pcg.st, 0, kRMax * sizeof(PcgState), st));
  // assembly (Gauss quadrature on the device)
  CK(assemble_saddle(pb->S, nu, pb->cpen, pb->rowptr, pb->col, pb->val, pb->diagQ, pb->w, st));
  hipLaunchKernelGGL(k_gather_diag, dim3(256), dim3(256), 0, st, pb->S.n_u, pb->Lrowptr, pb->Lsrc, pb->val, pb->diagA);
  CK(hipGetLastError());
  CK(convert<double, float>(pb->nnz, pb->val, pb->val32, st));
  // w . 1
  hipLaunchKernelGGL((k_pdot<1>), dim3(vec_blocks(pb->S.n_p)), dim3(kVT), 0, st, pb->S.n_p, int64_t(0), nullptr, pb->w,
                     pb->partials, pb->counter, pb->scratch);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(&pb->w1, pb->scratch, sizeof(double), hipMemcpyDeviceToHost, st));
  // IC(0) with the diagonal-shift retries
  {
    std::vector<int32_t>& lev = pb->lev_fwd;
    forward_levels(pb->L, pb->S.n_u, lev, &pb->nlev_fwd);
    pb->level_ptr.assign(pb->nlev_fwd + 1, 0);
    for (int64_t i = 0; i < pb->S.n_u; ++i) pb->level_ptr[lev[i] + 1]++;
    for (int l = 0; l < pb->nlev_fwd; ++l) pb->level_ptr[l + 1] += pb->level_ptr[l];
    std::vector<int32_t> rows(pb->S.n_u), fillp(pb->level_ptr.begin(), pb->level_ptr.end() - 1);
    for (int64_t i = 0; i < pb->S.n_u; ++i) rows[fillp[lev[i]]++] = int32_t(i);
    pb->level_rows = m.upload(rows, st);
    if (m.err != hipSuccess) return fail_hip(pb, m.err, "allocation", __LINE__);
    const double alphas[4] = {0.0, 1e-3, 1e-2, 1e-1};
    bool ok = false;
    for (int s = 0; s < 4 && !ok; ++s) {
      CK(ic0_factor(pb->S.n_u, pb->nnzL, pb->Lsrc, pb->Lrowptr, pb->Lcol, pb->val, alphas[s], pb->Lval,
                    pb->level_rows, pb->level_ptr, pb->flag, st));
      int fl = 0;
      CK(hipMemcpyAsync(&fl, pb->flag, sizeof(int), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      if (fl < 0) {
        ok = true;
        pb->ic_shift_steps = s;
      }
    }
    if (!ok) return fail(pb, STOKES_EBREAKDOWN, "IC(0) breakdown after the last diagonal shift");
  }
  // triangular-solve schedule for single right-hand sides
  {
    FactorSched& fs = pb->fsA;
    fs.L = &pb->L;
    fs.n = pb->S.n_u;
    fs.Lval = pb->Lval;
    fs.lev_fwd = &pb->lev_fwd;
    fs.lev_bwd = &pb->lev_bwd;
    fs.groups = [pb](int strip, std::vector<int32_t>& g, int* ng) { strip_groups(pb->S, strip, g, ng); };
    fs.blocks.assign(pb->S.voff, pb->S.voff + pb->S.dim + 1);  // the velocity components
    fs.helpers = kTrsvHelpers;
    SchedPair* sp = nullptr;
    int rc = get_schedule(pb, 1, false, &sp);
    if (rc) return rc;
    const int64_t sched_bytes = sp->fwd.fast.bytes64 + sp->bwd.fast.bytes64;
    pb->spmv_nt = sp->fwd.fast.ok && sched_bytes <= (int64_t(256) << 20);
  }
  // Mapped domain: the constant function's pressure coefficients kappa = Q^{-1} w and
  // w1 = w . kappa = |Omega|.  kappa spans the kernel of B^T, so every right-hand side's
  // pressure part is made orthogonal to it: it is solved to rounding, by CG preconditioned
  // with IC(0) of Q (Q's Cholesky factor for the polar map, where 1/J depends on xi_0 alone
  // and Q keeps its Kronecker structure; one or two iterations).
  if (pb->S.geom != 0) {
    int rc = ensure_pressure_ic0(pb);
    if (rc) return rc;
    Work* W = nullptr;
    if ((rc = get_work(pb, 1, false, &W))) return rc;
    pb->kappa = m.get<double>(pb->S.n_p);
    if (m.err != hipSuccess) return fail_hip(pb, m.err, "allocation", __LINE__);
    CK(hipMemsetAsync(pb->pcgQ.st, 0, sizeof(PcgState) * kRMax, st));
    rc = precond_pressure<double>(pb, *W, PQ_CG_IC0, pb->w, pb->kappa, pb->scratch + 102, nullptr, nullptr, 1e-15, 50);
    if (rc) return rc;
    CK(scale(pb->S.n_p, pb->kappa, 1.0 / (2.0 * nu), st));
    hipLaunchKernelGGL((k_pdot<1>), dim3(vec_blocks(pb->S.n_p)), dim3(kVT), 0, st, pb->S.n_p, int64_t(0), pb->w,
                       pb->kappa, pb->partials, pb->counter, pb->scratch);
    CK(hipGetLastError());
    CK(hipMemcpyAsync(&pb->w1, pb->scratch, sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
  }
  // MINRES convergence flags (pinned host words) and the no-allocation solve's events and
  // workspace address, so that stokes_solve_noalloc allocates nothing later
  CK(hipHostMalloc((void**)&pb->hflag, 2 * sizeof(int), hipHostMallocDefault));
  for (auto& e : pb->flag_ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& e : pb->noalloc_ev) CK(hipEventCreate(&e));
  if (dev < 0 || dev >= kMaxDevices) return fail(pb, STOKES_EINVAL, "device index out of range");
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
      void* ptr = nullptr;
      CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
      g_scratch_ptr[dev] = ptr;
    }
    pb->noalloc_ws = g_scratch_ptr[dev];
  }
  CK(hipStreamSynchronize(st));
  auto t1 = std::chrono::steady_clock::now();
  pb->setup_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  return 0;
}

int stokes_sizes(const stokes_problem* pb, int64_t* n_u, int64_t* n_p) {
  if (!pb) return STOKES_EINVAL;
  if (n_u) *n_u = pb->S.n_u;
  if (n_p) *n_p = pb->S.n_p;
  return 0;
}

int stokes_set_stream(stokes_problem* pb, void* s) {
  if (!pb) return STOKES_EINVAL;
  pb->stream = static_cast<hipStream_t>(s);
  return 0;
}

int stokes_set_nu(stokes_problem* pb, double nu) {
  if (!pb || !(nu > 0.0) || !std::isfinite(nu)) return fail(pb, STOKES_EINVAL, "nu must be positive");
  const double r = nu / pb->nu;
  hipStream_t st = pb->stream;
  hipLaunchKernelGGL(k_scale_A, dim3(1024), dim3(256), 0, st, pb->S.n_u, pb->rowptr, pb->aend, pb->val, r);
  CK(hipGetLastError());
  CK(scale(pb->nnzL, pb->Lval, std::sqrt(r), st));
  hipLaunchKernelGGL(k_gather_diag, dim3(256), dim3(256), 0, st, pb->S.n_u, pb->Lrowptr, pb->Lsrc, pb->val, pb->diagA);
  CK(hipGetLastError());
  CK(convert<double, float>(pb->nnz, pb->val, pb->val32, st));
  for (auto& sp : pb->fsA.scheds) {
    CK(launch_trsv_gather(sp->fwd, pb->Lval, st));
    CK(launch_trsv_gather(sp->bwd, pb->Lval, st));
  }
  CK(hipStreamSynchronize(st));
  pb->nu = nu;
  return 0;
}

int stokes_set_inner_tol(stokes_problem* pb, double rtol) {
  if (!pb) return STOKES_EINVAL;
  if (rtol > 0.0) pb->inner_tol = rtol;
  return 0;
}

int stokes_set_refine_tol(stokes_problem* pb, double rtol) {
  if (!pb) return STOKES_EINVAL;
  if (!(rtol < 1.0)) return fail(pb, STOKES_EINVAL, "refine_tol must be < 1");
  if (rtol > 0.0) pb->refine_tol = rtol;
  return 0;
}

int stokes_set_restarts(stokes_problem* pb, int max_cycles) {
  if (!pb) return STOKES_EINVAL;
  if (max_cycles < 0 || max_cycles > 30) return fail(pb, STOKES_EINVAL, "restarts must be in 0..30");
  pb->restarts = max_cycles;
  return 0;
}

int stokes_set_maxit(stokes_problem* pb, int outer, int inner) {
  if (!pb) return STOKES_EINVAL;
  if (outer > 0) pb->maxit_outer = outer;
  if (inner > 0) pb->maxit_inner = inner;
  return 0;
}

int stokes_load(stokes_problem* pb, const stokes_forcing* spec, int nrhs, double* f_dev) {
  if (!pb || !spec || !f_dev || nrhs < 1) return fail(pb, STOKES_EINVAL, "bad arguments to stokes_load");
  const int M = spec->nmodes;
  if (M < 0 || M > 64 || (M > 0 && (!spec->amp || !spec->wave || !spec->phase)))
    return fail(pb, STOKES_EINVAL, "bad forcing mode tables");
  const int dim = pb->S.dim;
  DevAlloc tmp;
  double* amp = tmp.get<double>(size_t(nrhs) * dim * std::max(M, 1));
  int32_t* wave = tmp.get<int32_t>(size_t(nrhs) * dim * std::max(M, 1));
  double* phase = tmp.get<double>(size_t(nrhs) * dim * std::max(M, 1));
  if (tmp.err != hipSuccess) {
    tmp.release();
    return fail_hip(pb, tmp.err, "stokes_load allocation", __LINE__);
  }
  hipStream_t st = pb->stream;
  if (M > 0) {
    CK(hipMemcpyAsync(amp, spec->amp, sizeof(double) * nrhs * dim * M, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(wave, spec->wave, sizeof(int32_t) * nrhs * dim * M, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(phase, spec->phase, sizeof(double) * nrhs * dim * M, hipMemcpyHostToDevice, st));
  }
  hipError_t e = assemble_load(pb->S, pb->nu, spec->manufactured, M, nrhs, amp, wave, phase, f_dev, st);
  tmp.release();
  if (e != hipSuccess) return fail_hip(pb, e, "assemble_load", __LINE__);
  return 0;
}

int stokes_load_cavity(stokes_problem* pb, int kind, double* f_dev) {
  if (pb && pb->S.geom != 0) return fail(pb, STOKES_EINVAL, "stokes_load_cavity: the cavity is the unit square");
  if (!pb || !f_dev) return fail(pb, STOKES_EINVAL, "bad arguments to stokes_load_cavity");
  if (pb->S.dim != 2) return fail(pb, STOKES_EINVAL, "stokes_load_cavity: 2D problems only");
  if (kind != STOKES_CAVITY_LID && kind != STOKES_CAVITY_VERIFY)
    return fail(pb, STOKES_EINVAL, "stokes_load_cavity: unknown kind");
  hipError_t e = assemble_load_cavity(pb->S, pb->nu, pb->cpen, kind, f_dev, pb->stream);
  if (e != hipSuccess) return fail_hip(pb, e, "assemble_load_cavity", __LINE__);
  return 0;
}

int stokes_solve_batched(stokes_problem* pb, int nrhs, const double* F, double* U, double* P, double tol, int precond,
                         int precision, stokes_info* infos) {
  if (!pb) return STOKES_EINVAL;
  if (nrhs < 1 || nrhs > kRMax) return fail(pb, STOKES_EINVAL, "nrhs must be in 1..16");
  int rc = check_args_solve(pb, tol, precond, precision);
  if (rc) return rc;
  if ((rc = validate_vec(pb, F, "F")) || (rc = validate_vec(pb, U, "U")) || (rc = validate_vec(pb, P, "P"))) return rc;
  const int R = round_r(nrhs);
  Work* W = nullptr;
  if ((rc = get_work(pb, R, false, &W))) return rc;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n_p = pb->S.n_p, n = n_u + n_p;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, st, int64_t(n * R), (double*)W->b, 0.0);
  CK(hipGetLastError());
  // columns 0..nrhs-1 of F into the velocity rows; pressure rows stay zero
  if (R == nrhs) {
    CK(to_interleaved<double, double>(R, n_u, F, n_u, (double*)W->b, 0, st));
  } else {
    for (int c = 0; c < nrhs; ++c)
      CK(hipMemcpy2DAsync((double*)W->b + c, sizeof(double) * R, F + size_t(c) * n_u, sizeof(double), sizeof(double),
                          n_u, hipMemcpyDeviceToDevice, st));
  }
  if ((rc = check_finite(pb, R, (const double*)W->b, n))) return rc;
  rc = solve_core(pb, *W, precond, precision, tol, infos, nrhs);
  if (rc < 0) return rc;
  const int rc_solve = rc;
  if (R == nrhs) {
    CK(from_interleaved<double, double>(R, n_u, (const double*)W->x, 0, U, n_u, st));
    CK(from_interleaved<double, double>(R, n_p, (const double*)W->x, n_u, P, n_p, st));
  } else {
    for (int c = 0; c < nrhs; ++c) {
      CK(hipMemcpy2DAsync(U + size_t(c) * n_u, sizeof(double), (const double*)W->x + c, sizeof(double) * R,
                          sizeof(double), n_u, hipMemcpyDeviceToDevice, st));
      CK(hipMemcpy2DAsync(P + size_t(c) * n_p, sizeof(double), (const double*)W->x + size_t(n_u) * R + c,
                          sizeof(double) * R, sizeof(double), n_p, hipMemcpyDeviceToDevice, st));
    }
  }
  CK(hipEventRecord(e1, st));
  CK(hipEventSynchronize(e1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (infos)
    for (int c = 0; c < nrhs; ++c) infos[c].solve_ms = ms;
  return rc_solve;
}

int stokes_solve_noalloc(stokes_problem* pb, const double* f, double* u, double* pr, double tol, int precond,
                         stokes_info* info) {
  if (!pb) return STOKES_EINVAL;
  int rc = check_args_solve(pb, tol, precond, STOKES_FP64);
  if (rc) return rc;
  if (precond != STOKES_PC_IC0 && precond != STOKES_PC_JACOBI)
    return fail(pb, STOKES_EINVAL, "stokes_solve_noalloc: precond must be STOKES_PC_IC0 or STOKES_PC_JACOBI");
  if ((rc = validate_vec(pb, f, "f")) || (rc = validate_vec(pb, u, "u")) || (rc = validate_vec(pb, pr, "pr"))) return rc;
  const int64_t n_u = pb->S.n_u, n_p = pb->S.n_p, n = n_u + n_p;
  // every vector rounded up to 256 bytes
  const size_t vec_bytes = (size_t(n) * sizeof(double) + 255) & ~size_t(255);
  if (vec_bytes * kNoAllocVectors > kNoAllocBytes)
    return fail(pb, STOKES_EINVAL, "stokes_solve_noalloc: n_u + n_p exceeds the 64 MiB workspace (at most 838,848)");
  if (pb->noalloc_ws == nullptr || pb->hflag == nullptr || pb->noalloc_ev[0] == nullptr)
    return fail(pb, STOKES_EINVAL, "stokes_solve_noalloc: the handle was not set up by this library version");
  if (precond == STOKES_PC_IC0) {
    bool have = false;
    for (auto& sp : pb->fsA.scheds) have |= sp->rmax64 >= 1;
    if (!have) return fail(pb, STOKES_EINVAL, "stokes_solve_noalloc: no single-column FP64 triangular-solve schedule");
  }
  unsigned char* base = static_cast<unsigned char*>(pb->noalloc_ws);
  Work W;
  W.R = 1;
  W.fp32 = false;
  void** slots[kNoAllocVectors] = {&W.v[0], &W.v[1], &W.z[0], &W.z[1], &W.w[0], &W.w[1], &W.x, &W.q, &W.b, &W.y};
  for (int k = 0; k < kNoAllocVectors; ++k) *slots[k] = base + size_t(k) * vec_bytes;
  // kernel timing would create events on demand: off for this call
  const bool prof_was = pb->prof_on;
  pb->prof_on = false;
  hipStream_t st = pb->stream;
  CK(hipEventRecord(pb->noalloc_ev[0], st));
  // right-hand side [f; 0] (the array keeps the previous call's contents: every vector the
  // solve reads before writing is set here or by the MINRES initialisation)
  hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, st, n, (double*)W.b, 0.0);
  CK(hipGetLastError());
  CK(hipMemcpyAsync(W.b, f, sizeof(double) * n_u, hipMemcpyDeviceToDevice, st));
  rc = check_finite(pb, 1, (const double*)W.b, n);
  if (rc == 0) rc = solve_core(pb, W, precond, STOKES_FP64, tol, info, 1);
  pb->prof_on = prof_was;
  if (rc < 0) return rc;
  CK(hipMemcpyAsync(u, W.x, sizeof(double) * n_u, hipMemcpyDeviceToDevice, st));
  CK(hipMemcpyAsync(pr, (const double*)W.x + n_u, sizeof(double) * n_p, hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(pb->noalloc_ev[1], st));
  CK(hipEventSynchronize(pb->noalloc_ev[1]));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, pb->noalloc_ev[0], pb->noalloc_ev[1]));
  if (info) info->solve_ms = ms;
  return rc;
}

int stokes_solve_precision(stokes_problem* pb, const double* f, double* u, double* pr, double tol, int precond,
                           int precision, stokes_info* info) {
  return stokes_solve_batched(pb, 1, f, u, pr, tol, precond, precision, info);
}

int stokes_solve(stokes_problem* pb, const double* f, double* u, double* pr, double tol, int precond,
                 stokes_info* info) {
  return stokes_solve_batched(pb, 1, f, u, pr, tol, precond, STOKES_FP64, info);
}

int stokes_solve_adjoint_batched(stokes_problem* pb, int nrhs, const double* G, double* Lambda, double tol, int precond,
                                 stokes_info* infos) {
  if (!pb) return STOKES_EINVAL;
  if (nrhs < 1 || nrhs > kRMax) return fail(pb, STOKES_EINVAL, "nrhs must be in 1..16");
  int rc = check_args_solve(pb, tol, precond, STOKES_FP64);
  if (rc) return rc;
  if ((rc = validate_vec(pb, G, "g")) || (rc = validate_vec(pb, Lambda, "lambda"))) return rc;
  const int R = round_r(nrhs);
  Work* W = nullptr;
  if ((rc = get_work(pb, R, false, &W))) return rc;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n_p = pb->S.n_p, n = n_u + n_p;
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  CK(hipEventRecord(e0, st));
  hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, st, int64_t(n * R), (double*)W->b, 0.0);
  CK(hipGetLastError());
  for (int c = 0; c < nrhs; ++c)
    CK(hipMemcpy2DAsync((double*)W->b + c, sizeof(double) * R, G + size_t(c) * n, sizeof(double), sizeof(double), n,
                        hipMemcpyDeviceToDevice, st));
  if ((rc = check_finite(pb, R, (const double*)W->b, n))) return rc;
  // P^T g_p = g_p - w (kappa . g_p) / (w . kappa), kappa the constant's coefficients
  R_SWITCH(R, hipLaunchKernelGGL((k_pdot<RR>), dim3(vec_blocks(n_p)), dim3(kVT), 0, st, n_p, n_u, pb->kappa,
                                 (const double*)W->b, pb->partials, pb->counter, pb->scratch);
           hipLaunchKernelGGL((k_sub_w<RR>), dim3(256), dim3(256), 0, st, n_u, n_p, (double*)W->b, pb->w, pb->scratch,
                              pb->w1));
  CK(hipGetLastError());
  rc = solve_core(pb, *W, precond, STOKES_FP64, tol, infos, nrhs);
  if (rc < 0) return rc;
  const int rc_solve = rc;
  for (int c = 0; c < nrhs; ++c)
    CK(hipMemcpy2DAsync(Lambda + size_t(c) * n, sizeof(double), (const double*)W->x + c, sizeof(double) * R,
                        sizeof(double), n, hipMemcpyDeviceToDevice, st));
  CK(hipEventRecord(e1, st));
  CK(hipEventSynchronize(e1));
  float ms = 0.f;
  CK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (infos)
    for (int c = 0; c < nrhs; ++c) infos[c].solve_ms = ms;
  return rc_solve;
}

int stokes_solve_adjoint(stokes_problem* pb, const double* g, double* lambda, double tol, int precond,
                         stokes_info* info) {
  return stokes_solve_adjoint_batched(pb, 1, g, lambda, tol, precond, info);
}

int stokes_dnu_dot(stokes_problem* pb, int nrhs, const double* lam_u, const double* u, double* out) {
  if (!pb || nrhs < 1 || !lam_u || !u || !out) return fail(pb, STOKES_EINVAL, "bad arguments to stokes_dnu_dot");
  Work* W = nullptr;
  int rc = get_work(pb, 1, false, &W);
  if (rc) return rc;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u;
  // results go through scratch[0..kRMax) in chunks of kRMax right-hand sides
  for (int c0 = 0; c0 < nrhs; c0 += kRMax) {
    const int nc = std::min(kRMax, nrhs - c0);
    for (int c = 0; c < nc; ++c) {
      CK(spmv_resid<double>(1, pb->rs_A, pb->rowptr, pb->aend, pb->col, pb->val, u + size_t(c0 + c) * n_u, nullptr,
                            (double*)W->q, pb->partials, pb->counter, nullptr, st));
      CK(dot<double, double>(1, 0, n_u, lam_u + size_t(c0 + c) * n_u, (const double*)W->q, pb->partials, pb->counter,
                             pb->scratch + c, st));
    }
    double h[kRMax];
    CK(hipMemcpyAsync(h, pb->scratch, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (int c = 0; c < nc; ++c) out[c0 + c] = h[c] / pb->nu;
  }
  return 0;
}

int stokes_apply(stokes_problem* pb, const double* x, double* y) {
  if (!pb || !x || !y) return fail(pb, STOKES_EINVAL, "bad arguments to stokes_apply");
  const int64_t n = pb->S.n_u + pb->S.n_p;
  CK(spmv_resid<double>(1, pb->rs_full, pb->rowptr, nullptr, pb->col, pb->val, x, nullptr, y, pb->partials, pb->counter, nullptr,
                        pb->stream));
  CK(hipStreamSynchronize(pb->stream));
  return 0;
}

int stokes_apply_precond(stokes_problem* pb, int precond, const double* r, double* y, int* inner_iters) {
  if (!pb || !r || !y || precond < 0 || precond > 7) return fail(pb, STOKES_EINVAL, "bad arguments");
  if (inner_iters) *inner_iters = 0;
  Work* W = nullptr;
  int rc = get_work(pb, 1, false, &W);
  if (rc) return rc;
  hipStream_t st = pb->stream;
  const int64_t n_u = pb->S.n_u, n = n_u + pb->S.n_p;
  hipLaunchKernelGGL(k_apply_diag, dim3(1024), dim3(256), 0, st, n_u, n, r, y, pb->diagQ,
                     precond == STOKES_PC_JACOBI ? pb->diagA : nullptr, 2.0 * pb->nu);
  CK(hipGetLastError());
  if (precond != STOKES_PC_JACOBI) {
    SchedPair* sp = nullptr;
    const int qkind = pressure_kind(precond);
    const bool pq_cg = qkind >= 0;
    const bool jac = precond == STOKES_PC_JPCG || precond == STOKES_PC_IDEAL_A || precond == STOKES_PC_PCGAQ ||
                     precond == STOKES_PC_IDEAL;
    if (!jac && (rc = get_schedule(pb, 1, false, &sp))) return rc;
    if (precond != STOKES_PC_IC0) CK(hipMemsetAsync(pb->pcg.st, 0, sizeof(PcgState) * kRMax, st));
    rc = precond_velocity<double>(pb, precond, *W, sp, r, y, pb->scratch + 100, nullptr, nullptr, nullptr);
    if (rc) return rc;
    if (sp && (rc = check_trsv_err(pb, sp))) return rc;
    int qtotal = 0;
    if (pq_cg) {
      if ((rc = ensure_pressure_cg(pb))) return rc;
      CK(hipMemsetAsync(pb->pcgQ.st, 0, sizeof(PcgState) * kRMax, st));
      rc = precond_pressure<double>(pb, *W, qkind, r + n_u, y + n_u, pb->scratch + 101, nullptr, nullptr);
      if (rc) return rc;
      PcgState pq;
      CK(hipMemcpyAsync(&pq, pb->pcgQ.st, sizeof(PcgState), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      qtotal = pq.total;
    }
    if (inner_iters && precond != STOKES_PC_IC0) {
      PcgState ps;
      CK(hipMemcpyAsync(&ps, pb->pcg.st, sizeof(PcgState), hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      *inner_iters = ps.total + qtotal;
    }
  }
  CK(hipStreamSynchronize(st));
  return 0;
}

int stokes_export_csr(stokes_problem* pb, int which, int64_t* nnz, int64_t* rowptr, int32_t* col, double* val) {
  if (!pb || which < 0 || which > 2) return fail(pb, STOKES_EINVAL, "bad arguments to stokes_export_csr");
  if (which == 2) {
    int rc = ensure_pressure_ic0(pb);
    if (rc) return rc;
  }
  const auto& rp = which == 0 ? pb->P.rowptr : (which == 1 ? pb->L.rowptr : pb->LQ.rowptr);
  const auto& cl = which == 0 ? pb->P.col : (which == 1 ? pb->L.col : pb->LQ.col);
  if (nnz) *nnz = int64_t(cl.size());
  if (rowptr)
    for (size_t i = 0; i < rp.size(); ++i) rowptr[i] = rp[i];
  if (col) std::memcpy(col, cl.data(), cl.size() * sizeof(int32_t));
  if (val) {
    CK(hipMemcpyAsync(val, which == 0 ? pb->val : (which == 1 ? pb->Lval : pb->LQval), cl.size() * sizeof(double),
                      hipMemcpyDeviceToHost, pb->stream));
    CK(hipStreamSynchronize(pb->stream));
  }
  return 0;
}

int stokes_export_pressure_mass(stokes_problem* pb, double* diagQ, double* w) {
  if (!pb) return STOKES_EINVAL;
  if (diagQ) CK(hipMemcpyAsync(diagQ, pb->diagQ, sizeof(double) * pb->S.n_p, hipMemcpyDeviceToHost, pb->stream));
  if (w) CK(hipMemcpyAsync(w, pb->w, sizeof(double) * pb->S.n_p, hipMemcpyDeviceToHost, pb->stream));
  CK(hipStreamSynchronize(pb->stream));
  return 0;
}

int stokes_levels(const stokes_problem* pb, int* fwd_levels, int* bwd_levels) {
  if (!pb || pb->fsA.scheds.empty()) return STOKES_EINVAL;
  if (fwd_levels) *fwd_levels = pb->fsA.scheds[0]->fwd.nlevels;
  if (bwd_levels) *bwd_levels = pb->fsA.scheds[0]->bwd.nlevels;
  return 0;
}

int stokes_profile(stokes_problem* pb, int enable, double* ms, int64_t* counts) {
  if (!pb) return STOKES_EINVAL;
  CK(hipStreamSynchronize(pb->stream));
  prof_flush(pb);
  if (ms)
    for (int k = 0; k < 5; ++k) ms[k] = pb->prof_ms[k];
  if (counts)
    for (int k = 0; k < 5; ++k) counts[k] = pb->prof_cnt[k];
  if (enable == 1) {
    for (int k = 0; k < 5; ++k) {
      pb->prof_ms[k] = 0.0;
      pb->prof_cnt[k] = 0;
    }
    pb->prof_on = true;
  } else if (enable == 0) {
    pb->prof_on = false;
  }
  return 0;
}

const char* stokes_last_error(const stokes_problem* pb) { return pb ? pb->err.c_str() : "null problem handle"; }

void stokes_destroy(stokes_problem* pb) {
  if (!pb) return;
  hipStreamSynchronize(pb->stream);
  delete pb;
}

}  // extern "C"

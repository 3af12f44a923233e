// Internal declarations shared by the host orchestration and the HIP kernels of
// libstokes.so.  Not part of the public ABI (include/stokes.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

namespace stk {

// ---------------------------------------------------------------------------
// Discrete spaces (Sec. 3.2 of the paper): per velocity component c and direction
// d the number of retained 1D functions, their offset and degree.
// ---------------------------------------------------------------------------
struct Spaces {
  int N = 0, kp = 0, dim = 0, pdeg = 0;  // elements/dir, pressure degree k', dim, k'+1
  int vcnt[3][3] = {{0}};                // retained 1D functions of comp c in dir d
  int vshift[3][3] = {{0}};              // 1D index = local index + vshift (1 in dir c)
  int vdeg[3][3] = {{0}};                // 1D degree of comp c in dir d
  int64_t voff[4] = {0};                 // component offsets in the velocity numbering
  int64_t n_u = 0, n_p = 0;
  int nlo = 0, nhi = 0;                  // N + k', N + k' + 1 (1D function counts)
  int geom = 0;                          // 0: identity map; 1: polar 1/8 annulus (2D)
};

Spaces make_spaces(int N, int kp, int dim);

// Saddle-point CSR pattern: rows 0..n_u-1 velocity (A entries then B^T entries),
// rows n_u..n-1 pressure (B entries).  Also the end of the A part of each velocity row.
struct SaddlePattern {
  std::vector<int32_t> rowptr;  // [n+1]  (nnz < 2^31 is checked)
  std::vector<int32_t> col;     // [nnz]
  std::vector<int32_t> aend;    // [n_u] position where the B^T part of velocity row i starts
};

int build_saddle_pattern(const Spaces& S, SaddlePattern& P, std::string& err);

// Lower triangle of A (IC(0) pattern), diagonal last in each row; lsrc[k] = index of the
// entry in the saddle CSR values.
struct LowerPattern {
  std::vector<int32_t> rowptr, col;
  std::vector<int64_t> src;
};
void build_lower_pattern(const Spaces& S, const SaddlePattern& P, LowerPattern& L);

// ---------------------------------------------------------------------------
// Triangular-solve schedule (one direction).  Rows are split into groups (one
// workgroup each, all resident together).  Inside a group the rows are processed in
// dependency-level order in "steps" of at most kTrsvRPS rows of one level; the
// dependencies of a row are spread over kTrsvG lanes, E per lane.  Every dependency
// value is read from an LDS slot.  Slots are assigned by value lifetime (interval
// allocation over steps), so LDS holds only a window of levels: local values from the
// step that computes them to their last local use; values of rows owned by other
// groups ("halo") from a fixed look-ahead before their first use to their last use.
// ---------------------------------------------------------------------------
constexpr int kTrsvG = 8;                  // lanes per row
constexpr int kTrsvRPS = 64 / kTrsvG;      // rows per step (one compute wave)
constexpr int kTrsvThreads = 128;          // compute wavefront + halo wavefront
constexpr int kTrsvHaloLookahead = 16;     // steps before first use a halo slot is allocated
constexpr int kTrsvDummyGroups = 256;      // workgroups with their own padding-store words
constexpr int kLevelStride = 1 << 21;      // progress value = epoch * stride + level + 1

#ifndef STOKES_TRSV_HELPERS
#define STOKES_TRSV_HELPERS 2
#endif
constexpr int kTrsvHelpers = STOKES_TRSV_HELPERS;  // coupling-row groups per strip (2D solves)

// Value codes of schedule entries that are not factor entries: -1 padding (value 0), and
// for coupling rows the coefficient 1 of a coupling value in its row and the diagonal -1
// of a coupling row.
constexpr int64_t kTrsvValOne = -2;
constexpr int64_t kTrsvValMinusOne = -3;

struct TrsvSchedHost {
  int ngroups = 0, nsteps = 0, E = 0, nlevels = 0, nslots = 0, strip = 0;
  int max_deg = 0;
  int64_t nrows = 0;                       // rows of the factor
  int64_t ncpl = 0;                        // coupling rows (numbered nrows, nrows + 1, ...)
  std::vector<int32_t> cpl_row;            // [ncpl] the row whose coupling value it is
  std::vector<int32_t> grp_cpl;            // [ngroups] 1: the group computes coupling rows
  std::vector<int32_t> grp_step_ptr;       // [ngroups+1]
  std::vector<int32_t> grp_halo_ptr;       // [ngroups+1]
  std::vector<int32_t> halo_row;           // remote row (global index)
  std::vector<int32_t> halo_grp;           // producing group
  std::vector<int32_t> halo_lvl;           // level of the remote row
  std::vector<int32_t> halo_slot;          // LDS slot
  std::vector<int32_t> halo_free;          // steps (group-relative) that must be computed first
  std::vector<int32_t> step_level;         // [nsteps]
  std::vector<int32_t> step_halo_need;     // [nsteps] halo entries (prefix) that must be staged
  std::vector<int32_t> step_publish;       // [nsteps] 1: publish progress after this step
  std::vector<int32_t> srow;               // [nsteps*RPS] row or -1
  std::vector<int32_t> sslot;              // [nsteps*RPS] LDS slot of the result (0: not kept)
  std::vector<int64_t> sdiag_src;          // [nsteps*RPS] index of the diagonal in L values
  std::vector<int32_t> ent_src;            // [nsteps*E*64] LDS slot of the dependency
  std::vector<int64_t> ent_perm;           // [nsteps*E*64] index in L values or -1 (pad)
  std::vector<int32_t> ent_dep;            // [nsteps*E*64] the row read (checks), -1 (pad)
};

// Device layout of a schedule.  Per step the compute wave reads, per lane, EP factor
// values (EP = E rounded up to 4), EP 32-bit LDS slot ids and one 16-byte row record,
// all with vector loads, plus the global row (srow) and the per-solve right-hand side
// and dot-vector entries in schedule order.
struct TrsvRow64 {
  double dinv;   // reciprocal diagonal
  int32_t slot;  // LDS slot of the result (nslots, a dummy slot: not read later)
  int32_t need;  // halo entries (prefix) staged before the step (same for the step's rows)
};
struct TrsvRow32 {
  float dinv;
  int32_t slot;
  int32_t need;
  int32_t pad;
};
struct TrsvStep {
  int32_t level;    // dependency level of the step
  int32_t publish;  // 1: publish progress after this step
  int32_t need;     // halo entries (prefix) that must be staged
  int32_t pad;
};

// Single-column layout of a schedule (the launch of one right-hand side with a contiguous
// vector).  Each group has its own entries per lane, EP = 4 or 8 (the group's largest row
// over kTrsvG lanes), and its steps are stored as one block each, read with a single
// scalar base per step:
//   [kTrsvRPS row records (16 bytes)]
//   [64 lanes x EP LDS byte addresses (uint32)][64 lanes x EP factor values]
// A row record holds the reciprocal diagonal, the LDS byte address of the row's result
// slot, the row's byte offset in the output vector and the step's halo prefix (entries
// that must be staged before the step; the same in every record of a step), so that a
// step is five 16-byte loads per lane for EP = 4 (values 2, addresses 1, record 1, and the
// per-solve pair) and the prefetch window can hold more steps.  Steps with fewer than
// kTrsvRPS rows repeat their first row (the same arithmetic on the same data, so the
// repeated stores are identical), and every group is padded to a multiple of its prefetch
// depth with repeats of its last step; repeats add nothing to the fused dot product.  The
// per-solve right-hand side and dot-vector entries sit in a separate array of the same
// step order.
constexpr int kFastHdr = kTrsvRPS * 16;
template <typename T>
constexpr int fast_block_bytes(int ep) {
  return kFastHdr + 64 * ep * (4 + (int)sizeof(T));
}
#ifndef STOKES_FAST_DEPTH4
#define STOKES_FAST_DEPTH4 10
#endif
// register buffers of prefetched steps (EP = 4: 5 loads per step; EP = 8: 8), within the
// 63 vector-memory operations a wavefront can have outstanding
constexpr int fast_depth(int ep) { return ep == 4 ? STOKES_FAST_DEPTH4 : 6; }
constexpr int kFastMaxField = 65535;  // 16-bit LDS byte address and halo prefix (FP64 records)

struct FastRec64 {
  double dinv;
  uint32_t slot_need;  // LDS byte address of the result (low 16 bits), halo prefix (high 16)
  int32_t row_byte;
};
struct FastRec32 {
  float dinv;
  int32_t slot_byte;
  int32_t row_byte;
  int32_t need;
};

struct TrsvFastDev {
  bool ok = false;
  int nsteps = 0;                  // allocated steps (with padding and prefetch tail)
  int64_t bytes64 = 0;             // bytes of the FP64 blocks
  int32_t* grp_step_ptr = nullptr; // [ngroups+1] allocated step ranges
  int32_t* grp_npad = nullptr;     // [ngroups] executed steps (multiple of the group's depth)
  int32_t* grp_ep = nullptr;       // [ngroups] 4 or 8
  int64_t* grp_blk64 = nullptr;    // [ngroups+1] byte offset of the group's first block
  int64_t* grp_blk32 = nullptr;
  unsigned char* blk64 = nullptr;
  unsigned char* blk32 = nullptr;
  int64_t* step_val64 = nullptr;   // [nsteps] byte offset of each step's values (FP64 blocks)
  int64_t* step_val32 = nullptr;
  int32_t* step_ep = nullptr;      // [nsteps]
  int32_t* vperm = nullptr;        // [nsteps][64][8] index in L values or -1
  int32_t* dsrc = nullptr;         // [nsteps * RPS] index of the diagonal in L values
  int32_t* srow2 = nullptr;        // [nsteps * RPS] row, or ~row for a repeat (rows >= nrows:
                                   // coupling rows)
  void* dyn = nullptr;             // [nsteps * RPS] {rhs, dot} (16 bytes)
  // Groups and halo lists of this layout (its own: with coupling rows it has helper groups)
  int ngroups = 0, nslots = 0, nrows = 0, ncpl = 0;
  int32_t *grp_halo_ptr = nullptr, *halo_row = nullptr, *halo_slot = nullptr, *halo_free = nullptr;
  int32_t* grp_cpl = nullptr;      // [ngroups] 1: the group's rows are coupling rows
  void* cpl = nullptr;             // [ncpl] coupling values (FP64; FP32 solves use the front half)
  unsigned int* done_count = nullptr;
  double* partials = nullptr;      // [ngroups]
};

struct TrsvSchedDev {
  int ngroups = 0, nsteps = 0, E = 0, EP = 0, nlevels = 0, nslots = 0, nrows = 0;
  int64_t nent = 0;                // per-lane entries of all steps
  int32_t *grp_step_ptr = nullptr, *grp_halo_ptr = nullptr;
  int32_t* grp_ep = nullptr;       // [ngroups] entries per lane of the group's steps (4 or EP)
  int64_t* grp_eoff = nullptr;     // [ngroups+1] offset of the group's first step entries
  int32_t *halo_row = nullptr, *halo_grp = nullptr, *halo_lvl = nullptr, *halo_slot = nullptr, *halo_free = nullptr;
  int32_t* srow = nullptr;         // [nsteps*RPS] global row or -1 (rhs gather, writer)
  uint32_t* ssrc = nullptr;        // [nsteps][64][EP] LDS slot ids
  int64_t* vperm = nullptr;        // [nsteps][64][EP] index in L values or -1
  int64_t* dsrc = nullptr;         // [nsteps*RPS] index of the diagonal or -1
  TrsvStep* sstep = nullptr;       // [nsteps]
  double* sval = nullptr;          // [nsteps][64][EP] factor values in schedule order
  float* sval32 = nullptr;
  TrsvRow64* srinfo = nullptr;     // [nsteps*RPS]
  TrsvRow32* srinfo32 = nullptr;
  void* rhs_s = nullptr;           // rhs and dot vector in schedule order ([row slot][2][R_max] doubles)
  void* dummy = nullptr;           // targets of the stores of padding rows ([kTrsvDummyGroups][64] doubles)
  unsigned long long* progress = nullptr;  // [ngroups]
  unsigned long long* epoch = nullptr;     // [1]
  unsigned int* done_count = nullptr;      // [2]: one ticket per column block of a launch
  int* err = nullptr;                      // [1] spin-limit flag
  double* partials = nullptr;              // [ngroups * 16]
  void* cpl = nullptr;                     // [ncpl][kRMax] coupling rows' values (batched layout)
  int ncpl = 0;
  int rmax = 0;                            // widest R the LDS budget allows
  TrsvFastDev fast;                        // single-column layout (fast.ok)
};

// dir = +1 forward (L y = r), -1 backward (L^T z = y).  group_of[i] gives the group
// of each row (spatial strips).  Returns false with err on failure.
bool build_trsv_schedule(const LowerPattern& L, int64_t n, int dir, const std::vector<int32_t>& group_of,
                         int ngroups, TrsvSchedHost& S, std::string& err);

// The same with each row's dependencies on other blocks (blk: offsets of consecutive row
// blocks, solved in order) moved into coupling rows, one per (row, source block), computed
// by `helpers` extra groups per (group, source block).
bool build_trsv_schedule_coupled(const LowerPattern& L, int64_t n, int dir, const std::vector<int64_t>& blk,
                                 int helpers, const std::vector<int32_t>& group_of, int ngroups, TrsvSchedHost& S,
                                 std::string& err);

// Strip partition of the velocity rows: component c, last-direction 1D index t -> group
// offset_c + t / strip.
void strip_groups(const Spaces& S, int strip, std::vector<int32_t>& group_of, int* ngroups);

// Levels of the forward dependency DAG (used by the IC(0) factorisation too).
void forward_levels(const LowerPattern& L, int64_t n, std::vector<int32_t>& lev, int* nlev);

// ---------------------------------------------------------------------------
// Device-side MINRES scalar state (double buffered by iteration parity).
// ---------------------------------------------------------------------------
struct MinresState {
  double gamma, gamma_prev, gamma1, eta;
  double c, c_prev, s, s_prev;
  double delta, g2p, g2u, tolg;  // tolg = tol * gamma1
  int iter, done, status, maxit;
};

// Inner PCG state (IC(0)-PCG on A).
struct PcgState {
  double rho, pq, rr, bnorm2, rtol2;
  int iter, done, maxit, total;
};


// ---------------------------------------------------------------------------
// Krylov scalars on the device and the deterministic block reduction.
// ---------------------------------------------------------------------------
constexpr int kVT = 256;  // threads per block of the vector kernels
constexpr int kRMax = 16;

// Scalar arrays (device), indexed [parity][kind][column].
enum { RED_DELTA = 0, RED_G2P = 1, RED_G2U = 2, RED_KINDS = 3 };

struct MrScalars {
  MinresState* st;   // [2][kRMax]
  int* alldone;      // [2]
  double* red;       // [2][RED_KINDS][kRMax]
  double* partials;  // [kVecMaxBlocks * 2 * kRMax]
  unsigned int* counter;
};

__device__ __forceinline__ double* red_at(const MrScalars& s, int p, int kind) {
  return s.red + ((size_t)p * RED_KINDS + kind) * kRMax;
}

// Device-scope (coherent across the XCDs' L2 caches) relaxed loads and stores of 64/32-bit
// values, and a wait for this wave's outstanding vector memory operations (stores are
// acknowledged once visible device-wide).  Used instead of agent-scope fences, which
// write back or invalidate whole L2 caches.
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
__device__ __forceinline__ void wait_vm_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Block reduction of NV values per thread; the last block to finish (ticket) adds all
// block partials in a fixed order (thread t takes blocks t, t + kVT, ...; then a fixed
// tree) and calls fin(k, value) for k < NV on threads k < NV; returns true in that block.  Partials travel with
// device-scope stores and loads; a block takes its ticket only after its partial stores
// are acknowledged, so the last block sees every partial.
template <int NV, typename Fin>
__device__ bool reduce_last(double (&v)[NV], double* partials, unsigned int* counter, Fin fin) {
  static_assert(NV <= 64, "the partial stores and the ticket must come from one wavefront");
  __shared__ double sred[kVT / 64][NV];
  __shared__ int is_last;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) sred[wid][k] = x;
  }
  __syncthreads();
  if (tid < NV) {
    double x = 0.0;
#pragma unroll
    for (int w = 0; w < kVT / 64; ++w) x += sred[w][tid];
    dev_store(partials + (size_t)blockIdx.x * NV + tid, x);
  }
  if (tid == 0) {
    wait_vm_stores();  // wavefront 0 holds all NV partial stores
    const unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (unsigned int b = tid; b < gridDim.x; b += kVT)
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] += dev_load(partials + (size_t)b * NV + k);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) sred[wid][k] = x;
  }
  __syncthreads();
  if (tid < NV) {
    double x = 0.0;
#pragma unroll
    for (int w = 0; w < kVT / 64; ++w) x += sred[w][tid];
    fin(tid, x);
  }
  if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;  // this block ran fin
}

// Sum over aligned groups of SG lanes (SG = 8 or 16) with DPP row operations, on the
// 32-bit halves of a double: xor 1 and xor 2 inside quads, mirror inside half rows, then
// (SG = 16) mirror inside rows.
template <int CTRL>
__device__ __forceinline__ double dpp_mov64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)(unsigned)lo) | ((long long)hi << 32));
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov32(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov_any(double v) { return dpp_mov64<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ float dpp_mov_any(float v) { return dpp_mov32<CTRL>(v); }

template <int SG, typename T>
__device__ __forceinline__ T group_sum(T v) {
  v += dpp_mov_any<0xB1>(v);
  v += dpp_mov_any<0x4E>(v);
  v += dpp_mov_any<0x141>(v);
  if (SG == 16) v += dpp_mov_any<0x140>(v);
  return v;
}

// Grid of the elementwise kernels with a reduction: kVecItems items per thread, at most
// kVecMaxBlocks blocks
// (grid-stride loops).  Few blocks: the last-block reductions take one device-scope ticket
// per block, and the tickets serialise at about 10 ns each at the end of a short kernel
// (2D, N = 512: the Lanczos kernel took 45 us with 3,092 blocks for 30 MB, 21.7 us with
// 1,024).
#ifndef STOKES_VEC_ITEMS
#define STOKES_VEC_ITEMS 4
#endif
constexpr int kVecMaxBlocks = 1024;
constexpr int kVecItems = STOKES_VEC_ITEMS;
inline int vec_blocks(int64_t nitems, int items = kVecItems) {
  int64_t b = (nitems + int64_t(kVT) * items - 1) / (int64_t(kVT) * items);
  return int(std::max<int64_t>(1, std::min<int64_t>(b, kVecMaxBlocks)));
}
// Kernels without a reduction: one item per thread (more blocks in flight measured faster).
inline int vec_blocks_plain(int64_t nitems) { return vec_blocks(nitems, 1); }

struct PcgScalars {
  PcgState* st;     // [kRMax]
  int* alldone;     // [1]
  double* rho;      // [2][kRMax] (parity of the inner iteration)
  double* pq;       // [kRMax]
  double* rr;       // [kRMax]
  double* partials;
  unsigned int* counter;
};


// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
hipError_t assemble_saddle(const Spaces& S, double nu, double cpen, const int32_t* rowptr, const int32_t* col,
                           double* val, double* diagQ, double* w, hipStream_t st);
// Pressure mass matrix Q (CSR pattern given, values computed).
hipError_t assemble_Q(const Spaces& S, const int32_t* rowptr, const int32_t* col, double* val, hipStream_t st);
hipError_t assemble_load_cavity(const Spaces& S, double nu, double cpen, int kind, double* f, hipStream_t st);
hipError_t assemble_load(const Spaces& S, double nu, int manufactured, int nmodes, int nrhs, const double* amp_d,
                         const int32_t* wave_d, const double* phase_d, double* f, hipStream_t st);
hipError_t ic0_factor(int64_t n, int64_t nnzL, const int64_t* src, const int32_t* rowptr, const int32_t* col,
                      const double* Aval, double alpha, double* Lval, const int32_t* level_rows,
                      const std::vector<int32_t>& level_ptr, int* flag, hipStream_t st);
// Optional events recorded on the stream right before/after the solve kernel itself.
struct TrsvTiming {
  hipEvent_t before = nullptr, after = nullptr;
};
hipError_t launch_trsv(const TrsvSchedDev& S, bool fp32, int R, const void* rhs, void* out, const void* dotv,
                       double* dot_out, const int* skip, hipStream_t st, const TrsvTiming* tm = nullptr);
hipError_t launch_trsv_gather(const TrsvSchedDev& S, const double* Lval, hipStream_t st);
size_t trsv_shmem_bytes(int nslots, bool fp32, int R, bool compact = false);
// Static LDS of the solve kernels beside the dynamic part (the batched kernels' dot partials).
inline size_t trsv_static_shmem(int R) { return R >= 8 ? 256 : 0; }

// Row ranges of the CSR row kernels: block b owns rows split[b] .. split[b+1]-1 (device
// array of nb+1 entries), ranges balanced by entries on the host.
struct RowSplit {
  const int32_t* split = nullptr;
  int nb = 0;
};
constexpr int kSpmvBlocksPerCU = 8;
// Inner CG products (A rows, Q): their entries stay in the last-level cache between
// iterations, and fewer, longer blocks measured faster (2D N = 256, k' = 2, PCG(A,Q):
// 0.370 s at 8 blocks per CU, 0.338 s at 4 or 2; the saddle product is the same at 8, 4, 2).
constexpr int kPcgSpmvBlocksPerCU = 4;
std::vector<int32_t> balanced_row_split(const std::vector<int32_t>& rowptr, const std::vector<int32_t>* rowend,
                                        int64_t nrows, int nb);
int row_split_blocks(int64_t nrows, int num_cu, int per_cu = kSpmvBlocksPerCU);

template <typename T>
hipError_t mr_init_vec(int R, int64_t n, int64_t n_u, const T* b, T* v1, T* v0, T* w1, T* w0, T* x, T* z1,
                       const double* diagQ, const double* diagA, double two_nu, const MrScalars& s, hipStream_t st);
hipError_t mr_init_state(int R, const MrScalars& s, double tol, int maxit, hipStream_t st);
template <typename T>
// nt: read the matrix entries with non-temporal loads (they then leave the last-level cache to
// data that stays there, the triangular-solve schedules)
hipError_t mr_spmv(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* col, const T* val, const T* z, T* q,
                   const MrScalars& s, int p, bool nt, hipStream_t st);
template <typename T>
hipError_t mr_lanczos(int R, int64_t n, int64_t n_u, const T* q, const T* v, T* vprev_next, T* znext, const double* diagQ,
                      const double* diagA, double two_nu, const MrScalars& s, int p, hipStream_t st);
template <typename T>
hipError_t mr_update(int R, int64_t n, const T* z, const T* w, T* wprev_new, T* x, const MrScalars& s, int p,
                     hipStream_t st);
template <typename T>
hipError_t spmv_resid(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* rowend, const int32_t* col,
                      const T* val, const T* x, const T* b, T* y, double* partials, unsigned int* counter, double* out,
                      hipStream_t st);
template <typename Ta, typename Tb>
hipError_t dot(int R, int64_t r0, int64_t r1, const Ta* a, const Tb* b, double* partials, unsigned int* counter,
               double* out, hipStream_t st);
template <typename T>
// x_p -= (wp[c] / w1) kappa (kappa = nullptr: the all-ones vector, the identity map's constant)
hipError_t sub_mean(int R, int64_t n_u, int64_t n, T* x, const double* wp, double w1, const double* kappa,
                    hipStream_t st);
template <typename Ts, typename Td>
hipError_t to_interleaved(int R, int64_t len, const Ts* src, int64_t ld, Td* dst, int64_t dst_off, hipStream_t st);
template <typename Ts, typename Td>
hipError_t from_interleaved(int R, int64_t len, const Ts* src, int64_t src_off, Td* dst, int64_t ld, hipStream_t st);
template <typename Ts, typename Td>
hipError_t convert(int64_t n, const Ts* a, Td* b, hipStream_t st);
template <typename Td>
hipError_t accumulate(int R, int64_t nR, double* x, const Td* d, hipStream_t st);
hipError_t scale(int64_t n, double* a, double s, hipStream_t st);
template <typename T>
hipError_t scale_skip(int64_t n, T* a, double s, const int* skip, hipStream_t st);
template <typename T>
hipError_t pcg_init(int R, int64_t n_u, const T* b, T* r, T* x, const PcgScalars& s, const int* outer_done,
                    hipStream_t st);
template <typename T>
hipError_t pcg_init2(int R, int64_t n_u, const T* z, T* pv, const PcgScalars& s, double rtol, int maxit,
                     const int* outer_done, const MinresState* outer_st, hipStream_t st);
template <typename T>
hipError_t pcg_spmv(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* aend, const int32_t* col,
                    const T* val, const T* pv, T* q, const PcgScalars& s, bool stream_entries, hipStream_t st);
template <typename T>
hipError_t pcg_axpy(int R, int64_t n_u, const T* pv, const T* q, T* x, T* r, const PcgScalars& s, int ip,
                    hipStream_t st);
template <typename T>
hipError_t pcg_axpy_jacobi(int R, int64_t n, const T* pv, const T* q, const double* diag, T* x, T* r, T* z,
                           const PcgScalars& s, int ip, hipStream_t st);
template <typename T>
hipError_t pcg_pupdate(int R, int64_t n_u, const T* z, T* pv, const PcgScalars& s, int ip, hipStream_t st);
template <typename T>
hipError_t pcg_jacobi(int R, int64_t n_u, const T* r, const double* diag, T* z, const PcgScalars& s, double* rho_out,
                      const int* skip, hipStream_t st);


}  // namespace stk

// IC(0) factorisation of the velocity block A (Sec. 6.4 of the paper): L L^T ~ A with
// the sparsity of tril(A), row by row:
//   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj   (j < i in the pattern, increasing j)
//   L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)
// Rows of one dependency level are independent; one kernel launch per level, one
// wavefront per row.  The entries of row i stay in registers (two per lane, rows of up
// to 128 entries); the pattern and values of each row j it references are staged in
// LDS, where every lane looks up its own column by binary search.
#include "stokes_internal.h"

namespace stk {

constexpr int kIcMaxRow = 128;
constexpr int kIcWaves = 4;

// L values initialised from A, then the diagonal shift alpha * A_ii in a second launch
// (a diagonal entry is also an entry of the copy: one writer per launch).
__global__ void k_ic0_init(int64_t nnzL, const int64_t* __restrict__ src, const double* __restrict__ Aval,
                           double* __restrict__ Lval, int* __restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *flag = -1;
  if (k < nnzL) Lval[k] = Aval[src[k]];
}

__global__ void k_ic0_shift(const int64_t* __restrict__ src, const int32_t* __restrict__ Lrowptr, int64_t n,
                            const double* __restrict__ Aval, double alpha, double* __restrict__ Lval) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    const int64_t d = Lrowptr[k + 1] - 1;
    Lval[d] = Aval[src[d]] + alpha * Aval[src[d]];
  }
}

__global__ __launch_bounds__(64 * kIcWaves) void k_ic0_level(const int32_t* __restrict__ rows, int nrows,
                                                             const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ col,
                                                             double* __restrict__ Lval, int* __restrict__ flag) {
  __shared__ int32_t jcol[kIcWaves][kIcMaxRow];
  __shared__ double jval[kIcWaves][kIcMaxRow];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * kIcWaves + w;
  if (t >= nrows) return;
  const int i = rows[t];
  const int rb = rowptr[i], re = rowptr[i + 1];
  const int m = re - rb;  // entries of row i, diagonal last
  // row i entries: lane holds u = lane and u = lane + 64
  int c0 = -1, c1 = -1;
  double v0 = 0.0, v1 = 0.0;
  if (lane < m) {
    c0 = col[rb + lane];
    v0 = Lval[rb + lane];
  }
  if (lane + 64 < m) {
    c1 = col[rb + lane + 64];
    v1 = Lval[rb + lane + 64];
  }
  for (int u = 0; u < m - 1; ++u) {
    const int j = (u < 64) ? __shfl(c0, u, 64) : __shfl(c1, u - 64, 64);
    const double aij = (u < 64) ? __shfl(v0, u, 64) : __shfl(v1, u - 64, 64);
    const int jb = rowptr[j], je = rowptr[j + 1];
    const int mj = je - jb;
    if (lane < mj) {
      jcol[w][lane] = col[jb + lane];
      jval[w][lane] = Lval[jb + lane];
    }
    if (lane + 64 < mj) {
      jcol[w][lane + 64] = col[jb + lane + 64];
      jval[w][lane + 64] = Lval[jb + lane + 64];
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // sum over k < j present in row i (entries before u) and in row j (off-diagonal part)
    double prod = 0.0;
    for (int half = 0; half < 2; ++half) {
      const int uu = lane + 64 * half;
      const int ck = half ? c1 : c0;
      const double lik = half ? v1 : v0;
      if (uu < u) {
        int lo = 0, hi = mj - 2;  // search the off-diagonal entries of row j
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int cm = jcol[w][mid];
          if (cm == ck) {
            prod += lik * jval[w][mid];
            break;
          }
          if (cm < ck) lo = mid + 1;
          else hi = mid - 1;
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) prod += __shfl_xor(prod, off, 64);
    const double lij = (aij - prod) / jval[w][mj - 1];
    if (u < 64) {
      if (lane == u) v0 = lij;
    } else {
      if (lane == u - 64) v1 = lij;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
  // diagonal
  double sq = 0.0;
  if (lane < m - 1) sq += v0 * v0;
  if (lane + 64 < m - 1) sq += v1 * v1;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off, 64);
  const double ad = (m - 1 < 64) ? __shfl(v0, m - 1, 64) : __shfl(v1, m - 1 - 64, 64);
  const double dd = ad - sq;
  double ldiag = 0.0;
  if (dd > 0.0) {
    ldiag = sqrt(dd);
  } else if (lane == 0) {
    atomicMax(flag, i);
  }
  if (lane == m - 1) v0 = ldiag;
  if (lane + 64 == m - 1) v1 = ldiag;
  if (lane < m) Lval[rb + lane] = v0;
  if (lane + 64 < m) Lval[rb + lane + 64] = v1;
}

hipError_t ic0_factor(int64_t n, int64_t nnzL, const int64_t* src, const int32_t* rowptr, const int32_t* col,
                      const double* Aval, double alpha, double* Lval, const int32_t* level_rows,
                      const std::vector<int32_t>& level_ptr, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_ic0_init, dim3(unsigned((std::max<int64_t>(nnzL, 1) + 255) / 256)), dim3(256), 0, st, nnzL,
                     src, Aval, Lval, flag);
  if (alpha != 0.0)
    hipLaunchKernelGGL(k_ic0_shift, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, src, rowptr, n, Aval, alpha,
                       Lval);
  for (size_t l = 0; l + 1 < level_ptr.size(); ++l) {
    const int nr = level_ptr[l + 1] - level_ptr[l];
    if (nr == 0) continue;
    hipLaunchKernelGGL(k_ic0_level, dim3(unsigned((nr + kIcWaves - 1) / kIcWaves)), dim3(64 * kIcWaves), 0, st,
                       level_rows + level_ptr[l], nr, rowptr, col, Lval, flag);
  }
  return hipGetLastError();
}

}  // namespace stk

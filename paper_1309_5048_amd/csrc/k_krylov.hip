// Krylov kernels of the preconditioned MINRES solver (Sec. 5 of the paper) and of the
// inner IC(0)-PCG on A (Sec. 6.4), for R interleaved right-hand sides (vector layout
// [row][R]) in precision T (double, or float for the inner solve of the mixed mode).
//
// Scalars live on the device.  Reductions are deterministic: every block writes its
// partial sums, the last block to finish (atomic ticket) adds them in block order.
// The MINRES recurrence scalars are double buffered by iteration parity p: kernels of
// iteration j read state[p] and the update kernel writes state[1-p]; a per-parity
// "all columns done" flag makes every later kernel a no-op once all columns converged.
//
// MINRES iteration j (unnormalised z~_j = M^{-1} v_j, z_j = z~_j / gamma_j):
//   spmv    q = Acal z_j,  delta_j = q . z_j
//   lanczos v_{j+1} = q - (delta_j/gamma_j) v_j - (gamma_j/gamma_{j-1}) v_{j-1}
//           z~_{j+1,p} = 2 nu v_{j+1,p} / diag(Q)   (M_Q = Diag(Q)/(2 nu)); Jacobi M_A too
//   (velocity block: triangular solves / inner PCG, elsewhere)
//   update  gamma_{j+1} = sqrt(v_{j+1} . z~_{j+1}); Givens rotation; w, x updates.
#include "stokes_internal.h"

namespace stk {

// ---------------------------------------------------------------------------
// Sparse row products.  A row is handled by kSG lanes (kVT / kSG rows per block pass);
// each lane takes entries sub, sub + kSG, ... with U independent loads in flight, and the
// group adds its lanes with DPP row operations (every lane of the group gets the sum).
// Blocks take contiguous row ranges; when the grid is a multiple of 8 the ranges of the
// blocks that one XCD runs (blocks are dispatched round robin over the 8 XCDs) are
// adjacent, so the vector entries that an XCD gathers stay in its own L2.
// ---------------------------------------------------------------------------
constexpr int kSG = 16;
struct RowRange {
  int64_t begin, end;
};

// Rows of this block: the contiguous range split[b], split[b+1] (entries balanced on the
// host).  Blocks are dispatched round-robin over the 8 XCDs, so with a multiple of 8 blocks
// b is chosen such that the blocks of one XCD own adjacent ranges (their vector gathers
// then share that XCD's L2).
__device__ __forceinline__ RowRange block_rows(const int32_t* __restrict__ split) {
  const int nb = gridDim.x;
  const int b = (nb % 8 == 0) ? (int)(blockIdx.x % 8) * (nb / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  RowRange r;
  r.begin = split[b];
  r.end = split[b + 1];
  return r;
}

// R consecutive values (the R interleaved columns of one vector row) with wide loads.
template <int R, typename T>
__device__ __forceinline__ void load_cols(const T* __restrict__ p, T (&v)[R]) {
  if constexpr (R % 2 == 0 && sizeof(T) == 8) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) {
      const double2 t = q[c];
      v[2 * c] = t.x;
      v[2 * c + 1] = t.y;
    }
  } else if constexpr (R % 4 == 0 && sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int c = 0; c < R / 4; ++c) {
      const float4 t = q[c];
      v[4 * c] = t.x;
      v[4 * c + 1] = t.y;
      v[4 * c + 2] = t.z;
      v[4 * c + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) v[c] = p[c];
  }
}

// acc[c] = sum over k in [kb, ke) of val[k] * x[col[k] * R + c], in every lane of the group.
// Rows per lane group and entries per lane in the first chunk of a pass: with one column,
// two rows per group and 4 entries per lane (index, value and vector loads of both rows in
// flight at once); with R columns one row and fewer entries (register budget).
template <int R>
constexpr int spmv_rows_per_group() { return R == 1 ? 2 : 1; }
template <int R>
constexpr int spmv_chunk() { return R == 1 ? 4 : (R <= 8 ? 2 : 1); }
constexpr int kStageRows = 512;  // rows whose entry ranges a block stages in LDS at a time

// Entries [k0, k0 + U*kSG) of one row (lane sub takes k0 + sub + u*kSG), accumulated into
// acc with every load of the chunk issued before the first use.  Lanes past the row end
// load the row's last entry again and add nothing.
//
// The saddle product reads matrix entries with non-temporal loads: each product streams
// them once, and ordinary loads would let them (about 210 MB for the 2D N = 256, k' = 2
// system) evict the triangular-solve schedules from the last-level cache between products.
// Measured in a MINRES-IC(0) solve of that system: 412 -> 311 us per triangular solve,
// 62 -> 72 us per product.  The inner CG's product over the A rows takes either policy
// (NT): non-temporal beside the IC(0) schedules, ordinary where the A entries are the
// loop's whole working set and stay cached between its iterations.
// Matrix entry load: non-temporal (NT) or ordinary.
template <bool NT, typename T>
__device__ __forceinline__ T ld_entry(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

template <int R, int U, bool NT, typename Acc, typename T>
__device__ __forceinline__ void row_chunk(int32_t k0, int32_t ke, const int32_t* __restrict__ col,
                                          const T* __restrict__ val, const T* __restrict__ x, Acc (&acc)[R]) {
  int32_t j[U];
  T a[U];
  bool ok[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t k = k0 + u * kSG;
    ok[u] = k < ke;
    const int32_t kc = ok[u] ? k : ke - 1;
    j[u] = ld_entry<NT>(col + kc);
    a[u] = ld_entry<NT>(val + kc);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T xv[R];
    load_cols<R>(x + (size_t)j[u] * R, xv);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const Acc t = fma((Acc)a[u], (Acc)xv[c], acc[c]);
      acc[c] = ok[u] ? t : acc[c];
    }
  }
}

// Reduce-scatter of R = 8 or 16 columns over a row's kSG = 16 lanes: lane sub ends with the
// group's total of column scatter_col<R>(sub).  Each stage halves the columns a lane keeps
// (it keeps one half and adds the half its partner sends: mirror inside the row, mirror
// inside the half row, xor 2, xor 1); with 8 columns the last stage is a plain sum, so
// lanes sub and sub ^ 1 hold the same column.
template <int R>
__device__ __forceinline__ int scatter_col(int sub) {
  return (sub >= 8 ? R / 2 : 0) + ((sub & 7) >= 4 ? R / 4 : 0) + (((sub >> 1) & 1) ? R / 8 : 0) +
         ((sub & 1) ? R / 16 : 0);
}
template <int K, int CTRL, typename T>
__device__ __forceinline__ void scatter_stage(const T (&v)[2 * K], T (&o)[K], bool hi) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const T keep = hi ? v[K + i] : v[i];
    const T send = hi ? v[i] : v[K + i];
    o[i] = keep + dpp_mov_any<CTRL>(send);
  }
}
template <int R, typename T>
__device__ __forceinline__ T group_scatter(const T (&v)[R], int sub) {
  static_assert(kSG == 16 && (R == 8 || R == 16), "16 lanes, 8 or 16 columns");
  T a[R / 2], b[R / 4], c[R / 8];
  scatter_stage<R / 2, 0x140>(v, a, sub >= 8);
  scatter_stage<R / 4, 0x141>(a, b, (sub & 7) >= 4);
  scatter_stage<R / 8, 0x4E>(b, c, ((sub >> 1) & 1) != 0);
  if constexpr (R == 16) {
    T d[1];
    scatter_stage<1, 0xB1>(c, d, (sub & 1) != 0);
    return d[0];
  } else {
    return c[0] + dpp_mov_any<0xB1>(c[0]);
  }
}

// All rows of this block (entries rowptr[i] .. rowend[i]-1, or rowptr[i+1]-1 without
// rowend), kSG lanes per row and spmv_rows_per_group rows per lane group.  The rows' entry
// ranges are staged in LDS kStageRows at a time; the first chunk of every row of a pass is
// loaded together (one row chunk for each of the group's rows), longer rows continue row
// by row.  fin(i, acc) runs on lane 0 of the row's lane group with the row's sums; with kRS
// (R = 8 or 16) the group's lanes reduce-scatter the sums instead and fin(i, v, c) runs on
// every lane of the group with column c's sum v (lanes holding the same column call it
// with the same value).
template <int R, bool NT, typename Acc, bool kRS = false, typename T, typename Fin>
__device__ __forceinline__ void csr_rows(const int32_t* __restrict__ split, const int32_t* __restrict__ rowptr,
                                         const int32_t* __restrict__ rowend, const int32_t* __restrict__ col,
                                         const T* __restrict__ val, const T* __restrict__ x, Fin fin) {
  constexpr int RPG = spmv_rows_per_group<R>();
  constexpr int U = spmv_chunk<R>();
  constexpr int G = kVT / kSG;
  __shared__ int32_t s_kb[kStageRows], s_ke[kStageRows];
  const int sub = threadIdx.x & (kSG - 1);
  const int grp = threadIdx.x / kSG;
  const RowRange rr = block_rows(split);
  for (int64_t c0 = rr.begin; c0 < rr.end; c0 += kStageRows) {
    const int nrow = (int)min<int64_t>(kStageRows, rr.end - c0);
    for (int t = threadIdx.x; t < nrow; t += kVT) {
      s_kb[t] = rowptr[c0 + t];
      s_ke[t] = rowend ? rowend[c0 + t] : rowptr[c0 + t + 1];
    }
    __syncthreads();
    for (int base = 0; base < nrow; base += G * RPG) {
      int32_t kb[RPG], ke[RPG];
      Acc acc[RPG][R];
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        const int t = base + q * G + grp;
        kb[q] = t < nrow ? s_kb[t] : 0;
        ke[q] = t < nrow ? s_ke[t] : 0;
#pragma unroll
        for (int c = 0; c < R; ++c) acc[q][c] = Acc(0);
      }
      // first chunk of every row of the pass, all loads in flight together
      {
        int32_t j[RPG][U];
        T a[RPG][U];
        bool ok[RPG][U];
#pragma unroll
        for (int q = 0; q < RPG; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int32_t k = kb[q] + sub + u * kSG;
            ok[q][u] = k < ke[q];
            // (entry 0 for an empty or absent row: a valid address whose value is not added)
            const int32_t kc = ok[q][u] ? k : (ke[q] > kb[q] ? ke[q] - 1 : 0);
            j[q][u] = ld_entry<NT>(col + kc);
            a[q][u] = ld_entry<NT>(val + kc);
          }
#pragma unroll
        for (int q = 0; q < RPG; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            T xv[R];
            load_cols<R>(x + (size_t)j[q][u] * R, xv);
#pragma unroll
            for (int c = 0; c < R; ++c) {
              const Acc t = fma((Acc)a[q][u], (Acc)xv[c], acc[q][c]);
              acc[q][c] = ok[q][u] ? t : acc[q][c];
            }
          }
      }
      // the rest of longer rows
#pragma unroll
      for (int q = 0; q < RPG; ++q)
        for (int32_t k0 = kb[q] + sub + U * kSG; k0 < ke[q]; k0 += U * kSG) row_chunk<R, U, NT>(k0, ke[q], col, val, x, acc[q]);
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        const int t = base + q * G + grp;
        if constexpr (kRS) {
          const Acc v = group_scatter<R>(acc[q], sub);
          if (t < nrow) fin(c0 + t, v, scatter_col<R>(sub));
        } else {
#pragma unroll
          for (int c = 0; c < R; ++c) acc[q][c] = group_sum<kSG>(acc[q][c]);
          if (t < nrow && sub == 0) fin(c0 + t, acc[q]);
        }
      }
    }
    __syncthreads();
  }
}

// Store R consecutive values with wide stores.
template <int R, typename T>
__device__ __forceinline__ void store_cols(T* __restrict__ p, const T (&v)[R]) {
  if constexpr (R % 2 == 0 && sizeof(T) == 8) {
    double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
    for (int c = 0; c < R / 2; ++c) q[c] = double2{v[2 * c], v[2 * c + 1]};
  } else if constexpr (R % 4 == 0 && sizeof(T) == 4) {
    float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
    for (int c = 0; c < R / 4; ++c) q[c] = float4{v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
  } else {
#pragma unroll
    for (int c = 0; c < R; ++c) p[c] = v[c];
  }
}

// ---------------------------------------------------------------------------
// MINRES initialisation: v_1 = b, v_0 = w_0 = w_1 = x = 0, z~_1 pressure (and Jacobi
// velocity) part; gamma^2 partial sums of the pressure / velocity parts.
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_mr_init_vec(int64_t n, int64_t n_u, const T* __restrict__ b, T* __restrict__ v1,
                                                     T* __restrict__ v0, T* __restrict__ w1, T* __restrict__ w0,
                                                     T* __restrict__ x, T* __restrict__ z1, const double* __restrict__ diagQ,
                                                     const double* __restrict__ diagA, double two_nu, MrScalars s) {
  double acc[2 * R];
#pragma unroll
  for (int c = 0; c < 2 * R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVT) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const size_t k = (size_t)i * R + c;
      const T bv = b[k];
      v1[k] = bv;
      v0[k] = T(0);
      w1[k] = T(0);
      w0[k] = T(0);
      x[k] = T(0);
      if (i >= n_u) {
        const T zv = T(two_nu * (double)bv / diagQ[i - n_u]);
        z1[k] = zv;
        acc[c] += (double)bv * (double)zv;
      } else if (diagA != nullptr) {
        const T zv = T((double)bv / diagA[i]);
        z1[k] = zv;
        acc[R + c] += (double)bv * (double)zv;
      }
    }
  }
  reduce_last<2 * R>(acc, s.partials, s.counter, [&](int k, double val) {
    if (k < R) red_at(s, 0, RED_G2P)[k] = val;
    else if (diagA != nullptr) red_at(s, 0, RED_G2U)[k - R] = val;
  });
}

template <int R>
__global__ void k_mr_init_state(MrScalars s, double tol, int maxit) {
  const int c = threadIdx.x;
  __shared__ int nd;
  if (c == 0) nd = 0;
  __syncthreads();
  if (c < R) {
    const double g2 = red_at(s, 0, RED_G2P)[c] + red_at(s, 0, RED_G2U)[c];
    MinresState st;
    st.gamma_prev = 1.0;
    st.c = st.c_prev = 1.0;
    st.s = st.s_prev = 0.0;
    st.delta = st.g2p = st.g2u = 0.0;
    st.iter = 0;
    st.maxit = maxit;
    st.status = 0;
    st.done = 0;
    if (g2 < 0.0 || g2 != g2) {
      st.gamma = st.gamma1 = st.eta = 0.0;
      st.status = -4;
      st.done = 1;
    } else {
      st.gamma = st.gamma1 = st.eta = sqrt(g2);
      if (st.gamma1 == 0.0) st.done = 1;
    }
    st.tolg = tol * st.gamma1;
    if (maxit <= 0) st.done = 1;
    s.st[c] = st;
    s.st[kRMax + c] = st;
    if (st.done) atomicAdd(&nd, 1);
  }
  __syncthreads();
  if (c == 0) {
    s.alldone[0] = (nd == R);
    s.alldone[1] = (nd == R);
  }
}

// ---------------------------------------------------------------------------
// q = Acal z~_j / gamma_j and delta partials.
// ---------------------------------------------------------------------------
template <typename T, int R, bool NT>
__global__ __launch_bounds__(kVT) void k_mr_spmv(const int32_t* __restrict__ split, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ z, T* __restrict__ q, MrScalars s, int p) {
  if (s.alldone[p]) return;
  if constexpr (R > 1) {
    // the row's sums reduce-scattered over its 16 lanes: each lane finishes one column
    const int sub = threadIdx.x & (kSG - 1);
    const int cs = scatter_col<R>(sub);
    const bool lead = R == kSG || (sub & 1) == 0;  // one lane per column adds to the dot
    const MinresState& stc = s.st[p * kRMax + cs];
    const double igc = (stc.done || stc.gamma == 0.0) ? 0.0 : 1.0 / stc.gamma;
    double ad = 0.0;
    csr_rows<R, NT, T, true>(split, rowptr, nullptr, col, val, z, [&](int64_t i, T acc, int c) {
      const size_t k = (size_t)i * R + c;
      const T qv = T((double)acc * igc);
      if (lead) ad += (double)qv * (double)z[k] * igc;
      q[k] = qv;
    });
    double acc_d[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc_d[k] = k == cs ? ad : 0.0;
    reduce_last<R>(acc_d, s.partials, s.counter, [&](int k, double v) { red_at(s, p, RED_DELTA)[k] = v; });
    return;
  }
  double ig[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const MinresState& st = s.st[p * kRMax + c];
    ig[c] = (st.done || st.gamma == 0.0) ? 0.0 : 1.0 / st.gamma;
  }
  double acc_d[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc_d[c] = 0.0;
  csr_rows<R, NT, T>(split, rowptr, nullptr, col, val, z, [&](int64_t i, T (&acc)[R]) {
    T qv[R], zv[R];
    load_cols<R>(z + (size_t)i * R, zv);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      qv[c] = T((double)acc[c] * ig[c]);
      acc_d[c] += (double)qv[c] * (double)zv[c] * ig[c];
    }
    store_cols<R>(q + (size_t)i * R, qv);
  });
  reduce_last<R>(acc_d, s.partials, s.counter, [&](int k, double v) { red_at(s, p, RED_DELTA)[k] = v; });
}

// ---------------------------------------------------------------------------
// Lanczos update, pressure preconditioner (and Jacobi velocity preconditioner) and
// gamma^2 partial sums.  v_{j+1} overwrites v_{j-1}.
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_mr_lanczos(int64_t n, int64_t n_u, const T* __restrict__ q,
                                                    const T* __restrict__ v, T* __restrict__ vprev_next,
                                                    T* __restrict__ znext, const double* __restrict__ diagQ,
                                                    const double* __restrict__ diagA, double two_nu, MrScalars s,
                                                    int p) {
  if (s.alldone[p]) return;
  if constexpr (R > 1) {
    // one vector element (row i, column c) per thread: the grid stride is a multiple of R,
    // so a thread keeps its column and the loads of a wavefront are contiguous
    const int c = threadIdx.x % R;
    const MinresState& st = s.st[p * kRMax + c];
    const bool live = !st.done;
    const double ca = live ? red_at(s, p, RED_DELTA)[c] / st.gamma : 0.0;
    const double cb = live ? st.gamma / st.gamma_prev : 0.0;
    double ap = 0.0, au = 0.0;
    if (live)
      for (int64_t k = blockIdx.x * (int64_t)kVT + threadIdx.x; k < n * R; k += (int64_t)gridDim.x * kVT) {
        const int64_t i = k / R;
        const double vn = (double)q[k] - ca * (double)v[k] - cb * (double)vprev_next[k];
        const T vnt = T(vn);
        vprev_next[k] = vnt;
        if (i >= n_u) {
          const T zv = T(two_nu * (double)vnt / diagQ[i - n_u]);
          znext[k] = zv;
          ap += (double)vnt * (double)zv;
        } else if (diagA != nullptr) {
          const T zv = T((double)vnt / diagA[i]);
          znext[k] = zv;
          au += (double)vnt * (double)zv;
        }
      }
    double acc[2 * R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      acc[k] = k == c ? ap : 0.0;
      acc[R + k] = k == c ? au : 0.0;
    }
    reduce_last<2 * R>(acc, s.partials, s.counter, [&](int k, double val) {
      if (k < R) red_at(s, p, RED_G2P)[k] = val;
      else if (diagA != nullptr) red_at(s, p, RED_G2U)[k - R] = val;
    });
    return;
  }
  double ca[R], cb[R];
  bool live[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const MinresState& st = s.st[p * kRMax + c];
    live[c] = !st.done;
    const double dl = red_at(s, p, RED_DELTA)[c];
    ca[c] = live[c] ? dl / st.gamma : 0.0;
    cb[c] = live[c] ? st.gamma / st.gamma_prev : 0.0;
  }
  double acc[2 * R];
#pragma unroll
  for (int c = 0; c < 2 * R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVT) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (!live[c]) continue;
      const size_t k = (size_t)i * R + c;
      const double vn = (double)q[k] - ca[c] * (double)v[k] - cb[c] * (double)vprev_next[k];
      const T vnt = T(vn);
      vprev_next[k] = vnt;
      if (i >= n_u) {
        const T zv = T(two_nu * (double)vnt / diagQ[i - n_u]);
        znext[k] = zv;
        acc[c] += (double)vnt * (double)zv;
      } else if (diagA != nullptr) {
        const T zv = T((double)vnt / diagA[i]);
        znext[k] = zv;
        acc[R + c] += (double)vnt * (double)zv;
      }
    }
  }
  reduce_last<2 * R>(acc, s.partials, s.counter, [&](int k, double val) {
    if (k < R) red_at(s, p, RED_G2P)[k] = val;
    else if (diagA != nullptr) red_at(s, p, RED_G2U)[k - R] = val;
  });
}

// ---------------------------------------------------------------------------
// Givens rotation and w, x updates.  w_{j+1} overwrites w_{j-1}.  Block 0 writes the
// state of the next iteration (parity 1-p).
// ---------------------------------------------------------------------------
struct Givens {
  double gn, a1, a2, a3, cn, sn, eta_new, coef;
  int live, status;
};

__device__ __forceinline__ Givens givens_step(const MinresState& st, double delta, double g2) {
  Givens G;
  G.live = !st.done;
  G.status = 0;
  if (!G.live) {
    G.gn = G.a1 = G.a2 = G.a3 = G.cn = G.sn = G.eta_new = G.coef = 0.0;
    return G;
  }
  if (g2 < 0.0 || g2 != g2) {
    G.status = -4;
    g2 = 0.0;
  }
  G.gn = sqrt(g2);
  const double a0 = st.c * delta - st.c_prev * st.s * st.gamma;
  G.a1 = sqrt(a0 * a0 + G.gn * G.gn);
  G.a2 = st.s * delta + st.c_prev * st.c * st.gamma;
  G.a3 = st.s_prev * st.gamma;
  G.cn = a0 / G.a1;
  G.sn = G.gn / G.a1;
  G.coef = G.cn * st.eta;
  G.eta_new = -G.sn * st.eta;
  return G;
}

template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_mr_update(int64_t n, const T* __restrict__ z, const T* __restrict__ w,
                                                   T* __restrict__ wprev_new, T* __restrict__ x, MrScalars s, int p) {
  if (s.alldone[p]) {
    // frozen: carry the state to the next parity so later launches stay no-ops
    if (blockIdx.x == 0) {
      if (threadIdx.x < R) s.st[(1 - p) * kRMax + threadIdx.x] = s.st[p * kRMax + threadIdx.x];
      if (threadIdx.x == 0) s.alldone[1 - p] = 1;
    }
    return;
  }
  if constexpr (R > 1) {
    // one vector element per thread (the grid stride is a multiple of R: a thread keeps
    // its column)
    const int c = threadIdx.x % R;
    const MinresState& st = s.st[p * kRMax + c];
    const Givens G = givens_step(st, red_at(s, p, RED_DELTA)[c], red_at(s, p, RED_G2P)[c] + red_at(s, p, RED_G2U)[c]);
    const double ig = G.live ? 1.0 / st.gamma : 0.0;
    if (G.live)
      for (int64_t k = blockIdx.x * (int64_t)kVT + threadIdx.x; k < n * R; k += (int64_t)gridDim.x * kVT) {
        const double wn = ((double)z[k] * ig - G.a3 * (double)wprev_new[k] - G.a2 * (double)w[k]) / G.a1;
        wprev_new[k] = T(wn);
        x[k] = T((double)x[k] + G.coef * wn);
      }
  } else {
    const MinresState& st = s.st[p * kRMax];
    const Givens G = givens_step(st, red_at(s, p, RED_DELTA)[0], red_at(s, p, RED_G2P)[0] + red_at(s, p, RED_G2U)[0]);
    const double ig = G.live ? 1.0 / st.gamma : 0.0;
    if (G.live)
      for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVT) {
        const double wn = ((double)z[i] * ig - G.a3 * (double)wprev_new[i] - G.a2 * (double)w[i]) / G.a1;
        wprev_new[i] = T(wn);
        x[i] = T((double)x[i] + G.coef * wn);
      }
  }
  if (blockIdx.x == 0) {
    __shared__ int nd;
    if (threadIdx.x == 0) nd = 0;
    __syncthreads();
    if (threadIdx.x < R) {
      const int c = threadIdx.x;
      MinresState st = s.st[p * kRMax + c];
      // same rotation as G[c] (recomputed: a register array cannot be indexed by thread)
      const Givens g = givens_step(st, red_at(s, p, RED_DELTA)[c], red_at(s, p, RED_G2P)[c] + red_at(s, p, RED_G2U)[c]);
      if (g.live) {
        st.gamma_prev = st.gamma;
        st.gamma = g.gn;
        st.c_prev = st.c;
        st.c = g.cn;
        st.s_prev = st.s;
        st.s = g.sn;
        st.eta = g.eta_new;
        st.iter += 1;
        if (g.status != 0) {
          st.status = g.status;
          st.done = 1;
        } else if (fabs(st.eta) <= st.tolg || st.gamma == 0.0) {
          st.done = 1;
        } else if (st.iter >= st.maxit) {
          st.status = 1;
          st.done = 1;
        }
      }
      s.st[(1 - p) * kRMax + c] = st;
      if (st.done) atomicAdd(&nd, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) s.alldone[1 - p] = (nd == R);
  }
}

// ---------------------------------------------------------------------------
// Generic helpers
// ---------------------------------------------------------------------------
// y = Acal x (all rows) or, with bvec, y = b - Acal x; optional partial sums of y.y and b.b
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_spmv_resid(const int32_t* __restrict__ split, const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ rowend, const int32_t* __restrict__ col,
                                                    const T* __restrict__ val, const T* __restrict__ xin,
                                                    const T* __restrict__ bvec, T* __restrict__ y, double* partials,
                                                    unsigned int* counter, double* out /*[2][R] or null*/) {
  double acc_d[2 * R];
#pragma unroll
  for (int c = 0; c < 2 * R; ++c) acc_d[c] = 0.0;
  csr_rows<R, true, double>(split, rowptr, rowend, col, val, xin, [&](int64_t i, double (&acc)[R]) {
    T bv[R], yv[R];
    if (bvec) {
      load_cols<R>(bvec + (size_t)i * R, bv);
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c) bv[c] = T(0);
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const double y64 = bvec ? (double)bv[c] - acc[c] : acc[c];
      yv[c] = T(y64);
      acc_d[c] += y64 * y64;
      acc_d[R + c] += (double)bv[c] * (double)bv[c];
    }
    store_cols<R>(y + (size_t)i * R, yv);
  });
  if (out == nullptr) return;
  reduce_last<2 * R>(acc_d, partials, counter, [&](int k, double v) { out[k] = v; });
}

// out[c] = sum_i a[i,c] * b[i,c] over rows [r0, r1) (fixed-order reduction).
template <typename Ta, typename Tb, int R>
__global__ __launch_bounds__(kVT) void k_dot(int64_t r0, int64_t r1, const Ta* __restrict__ a, const Tb* __restrict__ b,
                                             double* partials, unsigned int* counter, double* out) {
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t i = r0 + blockIdx.x * (int64_t)kVT + threadIdx.x; i < r1; i += (int64_t)gridDim.x * kVT)
#pragma unroll
    for (int c = 0; c < R; ++c) acc[c] += (double)a[(size_t)i * R + c] * (double)b[(size_t)i * R + c];
  reduce_last<R>(acc, partials, counter, [&](int k, double v) { out[k] = v; });
}

// Zero-mean pressure: p_c -= (w . p_c) / (w . 1), rows [n_u, n).  mean computed by k_dot.
template <typename T, int R>
__global__ void k_sub_mean(int64_t n_u, int64_t n, T* __restrict__ x, const double* __restrict__ wp, double w1,
                           const double* __restrict__ kappa) {
  for (int64_t i = n_u + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (kappa == nullptr) {
#pragma unroll
      for (int c = 0; c < R; ++c) x[(size_t)i * R + c] = T((double)x[(size_t)i * R + c] - wp[c] / w1);
    } else {
      const double kv = kappa[i - n_u];
#pragma unroll
      for (int c = 0; c < R; ++c) x[(size_t)i * R + c] = T((double)x[(size_t)i * R + c] - (wp[c] / w1) * kv);
    }
  }
}

// Column-major [R][len] (stride ld) <-> interleaved [len][R], with type conversion.
template <typename Ts, typename Td, int R>
__global__ void k_to_interleaved(int64_t len, const Ts* __restrict__ src, int64_t ld, Td* __restrict__ dst,
                                 int64_t dst_off) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < len * R; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / R;
    const int c = int(t % R);
    dst[(size_t)(dst_off + i) * R + c] = Td(src[(size_t)c * ld + i]);
  }
}

template <typename Ts, typename Td, int R>
__global__ void k_from_interleaved(int64_t len, const Ts* __restrict__ src, int64_t src_off, Td* __restrict__ dst,
                                   int64_t ld) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < len * R; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / R;
    const int c = int(t % R);
    dst[(size_t)c * ld + i] = Td(src[(size_t)(src_off + i) * R + c]);
  }
}

template <typename Ts, typename Td>
__global__ void k_convert(int64_t n, const Ts* __restrict__ a, Td* __restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = Td(a[i]);
}

// x64 += d (any precision); both interleaved with the same R.
template <typename Td, int R>
__global__ void k_accumulate(int64_t nR, double* __restrict__ x, const Td* __restrict__ d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nR; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += (double)d[i];
}

__global__ void k_scale(int64_t n, double* __restrict__ a, double s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) a[i] *= s;
}

// ---------------------------------------------------------------------------
// Inner IC(0)-PCG on A (x0 = 0; stop when ||r||^2 <= rtol^2 ||b||^2, tested after each
// update; at most maxit iterations).  x aliases the velocity part of z~_{j+1}.
// ---------------------------------------------------------------------------

// r = b (velocity part of v_{j+1}), x = 0, ||b||^2
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_init(int64_t n_u, const T* __restrict__ b, T* __restrict__ r,
                                                  T* __restrict__ x, PcgScalars s, const int* outer_done) {
  if (outer_done != nullptr && *outer_done) return;
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * kVT)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const size_t k = (size_t)i * R + c;
      const T bv = b[k];
      r[k] = bv;
      x[k] = T(0);
      acc[c] += (double)bv * (double)bv;
    }
  reduce_last<R>(acc, s.partials, s.counter, [&](int k, double v) { s.rr[k] = v; });
}

// after z = M^{-1} r (rho[0] from the fused dot): p = z, state init
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_init2(int64_t n_u, const T* __restrict__ z, T* __restrict__ pv, PcgScalars s,
                                                   double rtol, int maxit, const int* outer_done,
                                                   const MinresState* outer_st) {
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n_u * R; i += (int64_t)gridDim.x * kVT) pv[i] = z[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int nd = 0;
    for (int c = 0; c < R; ++c) {
      PcgState st;
      st.rho = s.rho[c];
      st.bnorm2 = s.rr[c];
      st.rr = s.rr[c];
      st.rtol2 = rtol * rtol;
      st.pq = 0.0;
      st.iter = 0;
      st.maxit = maxit;
      st.total = s.st[c].total;
      st.done = (outer_done != nullptr && *outer_done) || (outer_st != nullptr && outer_st[c].done) ||
                st.bnorm2 == 0.0 || maxit <= 0;
      s.st[c] = st;
      nd += st.done;
    }
    *s.alldone = (nd == R);
  }
}

// q = A p (velocity rows, A part of the saddle CSR) and p.q partials
template <typename T, int R, bool NT>
__global__ __launch_bounds__(kVT) void k_pcg_spmv(const int32_t* __restrict__ split, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ aend, const int32_t* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ pv, T* __restrict__ q,
                                                  PcgScalars s) {
  if (*s.alldone) return;
  double acc_d[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc_d[c] = 0.0;
  csr_rows<R, NT, T>(split, rowptr, aend, col, val, pv, [&](int64_t i, T (&acc)[R]) {
    T pw[R];
    load_cols<R>(pv + (size_t)i * R, pw);
#pragma unroll
    for (int c = 0; c < R; ++c) acc_d[c] += (double)acc[c] * (double)pw[c];
    store_cols<R>(q + (size_t)i * R, acc);
  });
  reduce_last<R>(acc_d, s.partials, s.counter, [&](int k, double v) { s.pq[k] = v; });
}

// alpha = rho/pq; x += alpha p; r -= alpha q; ||r||^2 partials; last block: convergence
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_axpy(int64_t n_u, const T* __restrict__ pv, const T* __restrict__ q,
                                                  T* __restrict__ x, T* __restrict__ r, PcgScalars s, int ip) {
  if (*s.alldone) return;
  double al[R];
  bool live[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    live[c] = !s.st[c].done;
    al[c] = live[c] ? s.rho[ip * kRMax + c] / s.pq[c] : 0.0;
  }
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * kVT)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (!live[c]) continue;
      const size_t k = (size_t)i * R + c;
      x[k] = T((double)x[k] + al[c] * (double)pv[k]);
      const double rn = (double)r[k] - al[c] * (double)q[k];
      r[k] = T(rn);
      acc[c] += rn * rn;
    }
  const bool last = reduce_last<R>(acc, s.partials, s.counter, [&](int c, double v) {
    PcgState& st = s.st[c];
    if (!st.done) {
      st.rr = v;
      st.iter += 1;
      st.total += 1;
      if (v <= st.rtol2 * st.bnorm2 || st.iter >= st.maxit) st.done = 1;
    }
  });
  if (last) {  // the all-done flag, in the block that finished the reduction
    __syncthreads();
    if (threadIdx.x == 0) {
      int nd = 0;
      for (int c = 0; c < R; ++c) nd += s.st[c].done;
      *s.alldone = (nd == R);
    }
  }
}

// The CG update and the Jacobi step in one pass, for Diag-preconditioned CG: as k_pcg_axpy,
// then z = r / diag and rho = r.z into rho[1 - ip] for the live columns, both reductions
// in one (2R values).  Columns already done keep x, r and z.
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_axpy_jacobi(int64_t n, const T* __restrict__ pv,
                                                         const T* __restrict__ q, const double* __restrict__ diag,
                                                         T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                         PcgScalars s, int ip) {
  if (*s.alldone) return;
  double al[R];
  bool live[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    live[c] = !s.st[c].done;
    al[c] = live[c] ? s.rho[ip * kRMax + c] / s.pq[c] : 0.0;
  }
  double acc[2 * R];
#pragma unroll
  for (int c = 0; c < 2 * R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kVT) {
    const double d = diag[i];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (!live[c]) continue;
      const size_t k = (size_t)i * R + c;
      x[k] = T((double)x[k] + al[c] * (double)pv[k]);
      const double rn = (double)r[k] - al[c] * (double)q[k];
      const T rt = T(rn);
      r[k] = rt;
      acc[c] += rn * rn;
      const T zv = T((double)rt / d);
      z[k] = zv;
      acc[R + c] += (double)rt * (double)zv;
    }
  }
  const bool last = reduce_last<2 * R>(acc, s.partials, s.counter, [&](int k, double v) {
    if (k >= R) {
      s.rho[(1 - ip) * kRMax + (k - R)] = v;
      return;
    }
    PcgState& st = s.st[k];
    if (!st.done) {
      st.rr = v;
      st.iter += 1;
      st.total += 1;
      if (v <= st.rtol2 * st.bnorm2 || st.iter >= st.maxit) st.done = 1;
    }
  });
  if (last) {
    __syncthreads();
    if (threadIdx.x == 0) {
      int nd = 0;
      for (int c = 0; c < R; ++c) nd += s.st[c].done;
      *s.alldone = (nd == R);
    }
  }
}

// Jacobi preconditioner of the inner PCG: z = r / diag(A) and rho = r.z into rho_out[c]
// (the role of the fused dot of the IC(0) triangular solves).  skip: device flag or null.
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_jacobi(int64_t n_u, const T* __restrict__ r,
                                                    const double* __restrict__ diag, T* __restrict__ z,
                                                    double* __restrict__ partials, unsigned int* __restrict__ counter,
                                                    double* __restrict__ rho_out, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  double acc[R];
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * kVT) {
    const double d = diag[i];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const size_t k = (size_t)i * R + c;
      const T zv = T((double)r[k] / d);
      z[k] = zv;
      acc[c] += (double)r[k] * (double)zv;
    }
  }
  reduce_last<R>(acc, partials, counter, [&](int k, double v) { rho_out[k] = v; });
}

// beta = rho_new/rho; p = z + beta p  (rho_new in rho[1-ip])
template <typename T, int R>
__global__ __launch_bounds__(kVT) void k_pcg_pupdate(int64_t n_u, const T* __restrict__ z, T* __restrict__ pv,
                                                     PcgScalars s, int ip) {
  if (*s.alldone) return;
  double be[R];
  bool live[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    live[c] = !s.st[c].done;
    be[c] = live[c] ? s.rho[(1 - ip) * kRMax + c] / s.rho[ip * kRMax + c] : 0.0;
  }
  for (int64_t i = blockIdx.x * (int64_t)kVT + threadIdx.x; i < n_u; i += (int64_t)gridDim.x * kVT)
#pragma unroll
    for (int c = 0; c < R; ++c) {
      if (!live[c]) continue;
      const size_t k = (size_t)i * R + c;
      pv[k] = T((double)z[k] + be[c] * (double)pv[k]);
    }
}

// ===========================================================================
// Host launchers (explicit instantiation through switch on R)
// ===========================================================================
#define STK_R_SWITCH(R_, ...)                   \
  switch (R_) {                                 \
    case 1: { constexpr int RR = 1; __VA_ARGS__; break; } \
    case 8: { constexpr int RR = 8; __VA_ARGS__; break; } \
    case 16: { constexpr int RR = 16; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue;      \
  }

template <typename T>
hipError_t mr_init_vec(int R, int64_t n, int64_t n_u, const T* b, T* v1, T* v0, T* w1, T* w0, T* x, T* z1,
                       const double* diagQ, const double* diagA, double two_nu, const MrScalars& s, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_init_vec<T, RR>), dim3(vec_blocks(n)), dim3(kVT), 0, st, n, n_u, b, v1, v0, w1,
                                     w0, x, z1, diagQ, diagA, two_nu, s));
  return hipGetLastError();
}

hipError_t mr_init_state(int R, const MrScalars& s, double tol, int maxit, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_init_state<RR>), dim3(1), dim3(64), 0, st, s, tol, maxit));
  return hipGetLastError();
}

template <typename T>
hipError_t mr_spmv(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* col, const T* val, const T* z, T* q,
                   const MrScalars& s, int p, bool nt, hipStream_t st) {
  if (nt) {
    STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_spmv<T, RR, true>), dim3(rs.nb), dim3(kVT), 0, st, rs.split, rowptr, col,
                                       val, z, q, s, p));
  } else {
    STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_spmv<T, RR, false>), dim3(rs.nb), dim3(kVT), 0, st, rs.split, rowptr, col,
                                       val, z, q, s, p));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t mr_lanczos(int R, int64_t n, int64_t n_u, const T* q, const T* v, T* vprev_next, T* znext, const double* diagQ,
                      const double* diagA, double two_nu, const MrScalars& s, int p, hipStream_t st) {
  // batched: 16 elements per thread (fewer blocks, so fewer last-block tickets; C4 43 -> 33 us)
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_lanczos<T, RR>), dim3(vec_blocks(n * RR, RR > 1 ? 16 : kVecItems)), dim3(kVT), 0, st, n, n_u, q, v,
                                     vprev_next, znext, diagQ, diagA, two_nu, s, p));
  return hipGetLastError();
}

template <typename T>
hipError_t mr_update(int R, int64_t n, const T* z, const T* w, T* wprev_new, T* x, const MrScalars& s, int p,
                     hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_mr_update<T, RR>), dim3(vec_blocks_plain(n * RR)), dim3(kVT), 0, st, n, z, w, wprev_new, x,
                                     s, p));
  return hipGetLastError();
}

template <typename T>
hipError_t spmv_resid(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* rowend, const int32_t* col,
                      const T* val, const T* x, const T* b, T* y, double* partials, unsigned int* counter, double* out,
                      hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_spmv_resid<T, RR>), dim3(rs.nb), dim3(kVT), 0, st, rs.split, rowptr, rowend,
                                     col, val, x, b, y, partials, counter, out));
  return hipGetLastError();
}

template <typename Ta, typename Tb>
hipError_t dot(int R, int64_t r0, int64_t r1, const Ta* a, const Tb* b, double* partials, unsigned int* counter,
               double* out, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_dot<Ta, Tb, RR>), dim3(vec_blocks(r1 - r0)), dim3(kVT), 0, st, r0, r1, a, b,
                                     partials, counter, out));
  return hipGetLastError();
}

template <typename T>
hipError_t sub_mean(int R, int64_t n_u, int64_t n, T* x, const double* wp, double w1, const double* kappa,
                    hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_sub_mean<T, RR>), dim3(256), dim3(256), 0, st, n_u, n, x, wp, w1, kappa));
  return hipGetLastError();
}

template <typename Ts, typename Td>
hipError_t to_interleaved(int R, int64_t len, const Ts* src, int64_t ld, Td* dst, int64_t dst_off, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_to_interleaved<Ts, Td, RR>), dim3(1024), dim3(256), 0, st, len, src, ld, dst,
                                     dst_off));
  return hipGetLastError();
}

template <typename Ts, typename Td>
hipError_t from_interleaved(int R, int64_t len, const Ts* src, int64_t src_off, Td* dst, int64_t ld, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_from_interleaved<Ts, Td, RR>), dim3(1024), dim3(256), 0, st, len, src, src_off,
                                     dst, ld));
  return hipGetLastError();
}

template <typename Ts, typename Td>
hipError_t convert(int64_t n, const Ts* a, Td* b, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Ts, Td>), dim3(1024), dim3(256), 0, st, n, a, b);
  return hipGetLastError();
}

template <typename Td>
hipError_t accumulate(int R, int64_t nR, double* x, const Td* d, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_accumulate<Td, RR>), dim3(1024), dim3(256), 0, st, nR, x, d));
  return hipGetLastError();
}

// a *= s unless *skip (device flag or null)
template <typename T>
__global__ void k_scale_skip(int64_t n, T* __restrict__ a, double s, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = T((double)a[i] * s);
}

template <typename T>
hipError_t scale_skip(int64_t n, T* a, double s, const int* skip, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_skip<T>, dim3(1024), dim3(256), 0, st, n, a, s, skip);
  return hipGetLastError();
}
template hipError_t scale_skip<double>(int64_t, double*, double, const int*, hipStream_t);
template hipError_t scale_skip<float>(int64_t, float*, double, const int*, hipStream_t);

hipError_t scale(int64_t n, double* a, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(1024), dim3(256), 0, st, n, a, s);
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_init(int R, int64_t n_u, const T* b, T* r, T* x, const PcgScalars& s, const int* outer_done,
                    hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_init<T, RR>), dim3(vec_blocks(n_u)), dim3(kVT), 0, st, n_u, b, r, x, s,
                                     outer_done));
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_init2(int R, int64_t n_u, const T* z, T* pv, const PcgScalars& s, double rtol, int maxit,
                     const int* outer_done, const MinresState* outer_st, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_init2<T, RR>), dim3(vec_blocks(n_u * RR)), dim3(kVT), 0, st, n_u, z, pv, s,
                                     rtol, maxit, outer_done, outer_st));
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_spmv(int R, const RowSplit& rs, const int32_t* rowptr, const int32_t* aend, const int32_t* col,
                    const T* val, const T* pv, T* q, const PcgScalars& s, bool stream_entries, hipStream_t st) {
  if (stream_entries) {
    STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_spmv<T, RR, true>), dim3(rs.nb), dim3(kVT), 0, st, rs.split, rowptr,
                                       aend, col, val, pv, q, s));
  } else {
    STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_spmv<T, RR, false>), dim3(rs.nb), dim3(kVT), 0, st, rs.split, rowptr,
                                       aend, col, val, pv, q, s));
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_axpy_jacobi(int R, int64_t n, const T* pv, const T* q, const double* diag, T* x, T* r, T* z,
                           const PcgScalars& s, int ip, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_axpy_jacobi<T, RR>), dim3(vec_blocks(n)), dim3(kVT), 0, st, n, pv, q, diag,
                                     x, r, z, s, ip));
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_axpy(int R, int64_t n_u, const T* pv, const T* q, T* x, T* r, const PcgScalars& s, int ip,
                    hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_axpy<T, RR>), dim3(vec_blocks(n_u)), dim3(kVT), 0, st, n_u, pv, q, x, r, s,
                                     ip));
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_jacobi(int R, int64_t n_u, const T* r, const double* diag, T* z, const PcgScalars& s, double* rho_out,
                      const int* skip, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_jacobi<T, RR>), dim3(vec_blocks(n_u)), dim3(kVT), 0, st, n_u, r, diag, z,
                                     s.partials, s.counter, rho_out, skip));
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_pupdate(int R, int64_t n_u, const T* z, T* pv, const PcgScalars& s, int ip, hipStream_t st) {
  STK_R_SWITCH(R, hipLaunchKernelGGL((k_pcg_pupdate<T, RR>), dim3(vec_blocks_plain(n_u)), dim3(kVT), 0, st, n_u, z, pv, s, ip));
  return hipGetLastError();
}

// explicit instantiations used by the host code
#define STK_INST(T)                                                                                                   \
  template hipError_t mr_init_vec<T>(int, int64_t, int64_t, const T*, T*, T*, T*, T*, T*, T*, const double*,         \
                                     const double*, double, const MrScalars&, hipStream_t);                          \
  template hipError_t mr_spmv<T>(int, const RowSplit&, const int32_t*, const int32_t*, const T*, const T*, T*,      \
                                 const MrScalars&, int, bool, hipStream_t);                                         \
  template hipError_t mr_lanczos<T>(int, int64_t, int64_t, const T*, const T*, T*, T*, const double*, const double*,  \
                                    double, const MrScalars&, int, hipStream_t);                                     \
  template hipError_t mr_update<T>(int, int64_t, const T*, const T*, T*, T*, const MrScalars&, int, hipStream_t);    \
  template hipError_t spmv_resid<T>(int, const RowSplit&, const int32_t*, const int32_t*, const int32_t*, const T*,  \
                                    const T*, const T*, T*, double*, unsigned int*, double*, hipStream_t);           \
  template hipError_t sub_mean<T>(int, int64_t, int64_t, T*, const double*, double, const double*, hipStream_t);                    \
  template hipError_t pcg_init<T>(int, int64_t, const T*, T*, T*, const PcgScalars&, const int*, hipStream_t);       \
  template hipError_t pcg_init2<T>(int, int64_t, const T*, T*, const PcgScalars&, double, int, const int*,           \
                                   const MinresState*, hipStream_t);                                                 \
  template hipError_t pcg_spmv<T>(int, const RowSplit&, const int32_t*, const int32_t*, const int32_t*, const T*,    \
                                  const T*, T*, const PcgScalars&, bool, hipStream_t);                               \
  template hipError_t pcg_axpy<T>(int, int64_t, const T*, const T*, T*, T*, const PcgScalars&, int, hipStream_t);    \
  template hipError_t pcg_axpy_jacobi<T>(int, int64_t, const T*, const T*, const double*, T*, T*, T*,                \
                                         const PcgScalars&, int, hipStream_t);                                       \
  template hipError_t pcg_pupdate<T>(int, int64_t, const T*, T*, const PcgScalars&, int, hipStream_t);     \
  template hipError_t pcg_jacobi<T>(int, int64_t, const T*, const double*, T*, const PcgScalars&, double*,    \
                                    const int*, hipStream_t);
STK_INST(double)
STK_INST(float)

template hipError_t dot<double, double>(int, int64_t, int64_t, const double*, const double*, double*, unsigned int*,
                                        double*, hipStream_t);
template hipError_t dot<float, float>(int, int64_t, int64_t, const float*, const float*, double*, unsigned int*,
                                      double*, hipStream_t);
template hipError_t to_interleaved<double, double>(int, int64_t, const double*, int64_t, double*, int64_t, hipStream_t);
template hipError_t to_interleaved<double, float>(int, int64_t, const double*, int64_t, float*, int64_t, hipStream_t);
template hipError_t from_interleaved<double, double>(int, int64_t, const double*, int64_t, double*, int64_t,
                                                     hipStream_t);
template hipError_t convert<double, float>(int64_t, const double*, float*, hipStream_t);
template hipError_t convert<float, double>(int64_t, const float*, double*, hipStream_t);
template hipError_t accumulate<float>(int, int64_t, double*, const float*, hipStream_t);
template hipError_t accumulate<double>(int, int64_t, double*, const double*, hipStream_t);

}  // namespace stk

// CPU checks of the library's host-side integer logic (test support, not shipped):
//  * export of the closed-form saddle sparsity pattern, for comparison with the oracle;
//  * an emulator of the triangular-solve protocol (compute and halo wavefronts) that
//    executes a schedule with interleaved group progress and verifies, for every LDS read,
//    that the slot holds the value of the expected row (slot-lifetime allocation), that
//    halo values are staged only after their producer wrote them (the kernels poll for the
//    sentinel to be overwritten), that no wait can deadlock, and that every index is inside
//    its buffer; the result is compared with a direct triangular solve.  Schedules with
//    coupling rows (helper groups) are executed the same way, with the coupling values in
//    rows n, n + 1, ... of the output.
#include <cmath>
#include <cstdio>
#include <random>

#include "stokes_internal.h"

using namespace stk;

namespace {

struct Emu {
  int ok = 1;
  char msg[256] = {0};
  void bad(const char* m) {
    if (ok) snprintf(msg, sizeof(msg), "%s", m);
    ok = 0;
  }
};

// Execute schedule S (direction dir) for rhs b; returns x (natural order).
std::vector<double> emulate(const TrsvSchedHost& S, const LowerPattern& L, const std::vector<double>& Lval,
                            const std::vector<int32_t>& lrow, int64_t n, int dir, const std::vector<double>& b,
                            Emu& emu, long* rounds_out) {
  const int G = S.ngroups, E = S.E, RPS = kTrsvRPS;
  const int64_t nx = n + S.ncpl;  // rows with the coupling rows
  std::vector<double> out(nx, std::nan(""));
  std::vector<char> written(nx, 0);
  std::vector<int> k(G, 0), hpos(G, 0);
  std::vector<std::vector<double>> xs(G, std::vector<double>(S.nslots, std::nan("")));
  std::vector<std::vector<int32_t>> tag(G, std::vector<int32_t>(S.nslots, -2));
  for (int g = 0; g < G; ++g) {
    xs[g][0] = 0.0;
    tag[g][0] = -1;
  }
  long rounds = 0;
  for (;;) {
    bool moved = false, all_done = true;
    for (int g = 0; g < G; ++g) {
      const int s0 = S.grp_step_ptr[g], ns = S.grp_step_ptr[g + 1] - s0;
      const int h0 = S.grp_halo_ptr[g], nh = S.grp_halo_ptr[g + 1] - h0;
      // halo wave: stage the next ready entries in order
      while (hpos[g] < nh) {
        const int e = h0 + hpos[g];
        const int prod = S.halo_grp[e], lvl = S.halo_lvl[e], slot = S.halo_slot[e], row = S.halo_row[e];
        if (prod < 0 || prod >= G || slot <= 0 || slot >= S.nslots || row < 0 || row >= nx) {
          emu.bad("halo entry out of range");
          return out;
        }
        (void)lvl;
        if (!(written[row] && k[g] >= S.halo_free[e])) break;
        xs[g][slot] = out[row];
        tag[g][slot] = row;
        ++hpos[g];
        moved = true;
      }
      // compute wave: next step if its halo prefix is staged
      if (k[g] < ns) {
        all_done = false;
        const int ss = s0 + k[g];
        if (hpos[g] >= S.step_halo_need[ss]) {
          for (int r = 0; r < RPS; ++r) {
            const int row = S.srow[size_t(ss) * RPS + r];
            if (row < 0) continue;
            if (row >= nx || (row >= n) != (S.grp_cpl[g] != 0)) {
              emu.bad("step row out of range");
              return out;
            }
            double acc = 0.0;
            for (int e = 0; e < E; ++e)
              for (int q = 0; q < kTrsvG; ++q) {
                const size_t off = (size_t(ss) * E + e) * 64 + r * kTrsvG + q;
                const int src = S.ent_src[off];
                const int64_t perm = S.ent_perm[off];
                if (src < 0 || src >= S.nslots) {
                  emu.bad("entry slot out of range");
                  return out;
                }
                if (perm == -1) {
                  if (src != 0) emu.bad("padding entry not on the zero slot");
                  continue;
                }
                const int32_t dep = S.ent_dep[off];
                double coef;
                if (perm == kTrsvValOne) {
                  // a coupling value of this row
                  if (row >= n || dep < n || dep >= nx || S.cpl_row[dep - n] != row) {
                    emu.bad("coupling entry that is not one of the row's coupling rows");
                    return out;
                  }
                  coef = 1.0;
                } else if (perm >= 0 && perm < int64_t(Lval.size())) {
                  if (dep != (dir > 0 ? L.col[perm] : lrow[perm])) {
                    emu.bad("entry value and dependency disagree");
                    return out;
                  }
                  coef = Lval[perm];
                } else {
                  emu.bad("entry value index out of range");
                  return out;
                }
                if (tag[g][src] != dep) {
                  emu.bad("LDS slot does not hold the expected dependency (slot reuse or unstaged halo)");
                  return out;
                }
                acc += coef * xs[g][src];
              }
            const int64_t dsrc = S.sdiag_src[size_t(ss) * RPS + r];
            const bool is_cpl = row >= n;
            if (is_cpl != (dsrc == kTrsvValMinusOne)) {
              emu.bad("coupling row without the diagonal -1, or the reverse");
              return out;
            }
            const double x = ((is_cpl ? 0.0 : b[row]) - acc) / (is_cpl ? -1.0 : Lval[dsrc]);
            const int slot = S.sslot[size_t(ss) * RPS + r];
            if (slot < 0 || slot >= S.nslots) {
              emu.bad("result slot out of range");
              return out;
            }
            if (slot > 0) {
              xs[g][slot] = x;
              tag[g][slot] = row;
            }
            out[row] = x;
            written[row] = 1;
          }
          ++k[g];
          moved = true;
        }
      }
    }
    ++rounds;
    if (all_done) break;
    if (!moved) {
      emu.bad("deadlock: no group can make progress");
      return out;
    }
  }
  *rounds_out = rounds;
  return out;
}

}  // namespace

extern "C" {

// Saddle pattern of the library (closed form).  Call with null arrays to get sizes.
int hc_pattern(int N, int kp, int dim, int64_t* n_u, int64_t* n_p, int64_t* nnz, int64_t* rowptr, int32_t* col,
               int64_t* aend) {
  Spaces S = make_spaces(N, kp, dim);
  SaddlePattern P;
  std::string err;
  if (build_saddle_pattern(S, P, err) != 0) return -1;
  *n_u = S.n_u;
  *n_p = S.n_p;
  *nnz = int64_t(P.col.size());
  if (rowptr)
    for (size_t i = 0; i < P.rowptr.size(); ++i) rowptr[i] = P.rowptr[i];
  if (col)
    for (size_t i = 0; i < P.col.size(); ++i) col[i] = P.col[i];
  if (aend)
    for (size_t i = 0; i < P.aend.size(); ++i) aend[i] = P.aend[i];
  return 0;
}

// Build both schedules for a strip partition and emulate them on a random factor
// (helpers > 0: with coupling rows for the dependencies on other velocity components, that
// many helper groups per strip and source component).
// stats: [0] fwd levels [1] bwd levels [2] groups [3] fwd steps [4] bwd steps [5] max slots
//        [6] E [7] max rel error fwd [8] max rel error bwd [9] rounds fwd [10] rounds bwd
//        [11] halo entries fwd [12] max deps per row [13] coupling rows fwd
int hc_schedule_check(int N, int kp, int dim, int strip, int seed, int helpers, double* stats, char* msg,
                      int msglen) {
  Spaces S = make_spaces(N, kp, dim);
  SaddlePattern P;
  std::string err;
  if (build_saddle_pattern(S, P, err) != 0) return -1;
  LowerPattern L;
  build_lower_pattern(S, P, L);
  const int64_t n = S.n_u;
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> Lval(L.col.size());
  std::vector<int32_t> lrow(L.col.size());
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1]; ++k) {
      lrow[k] = int32_t(i);
      Lval[k] = (k == L.rowptr[i + 1] - 1) ? 4.0 + U(rng) : 0.1 * U(rng) / (L.rowptr[i + 1] - L.rowptr[i]);
    }
  std::vector<double> b(n);
  for (auto& v : b) v = U(rng);
  std::vector<int32_t> group_of;
  int ngroups = 0;
  strip_groups(S, strip, group_of, &ngroups);
  TrsvSchedHost F, B;
  std::vector<int64_t> blk(S.voff, S.voff + dim + 1);  // the velocity components
  if (helpers > 0 ? (!build_trsv_schedule_coupled(L, n, +1, blk, helpers, group_of, ngroups, F, err) ||
                     !build_trsv_schedule_coupled(L, n, -1, blk, helpers, group_of, ngroups, B, err))
                  : (!build_trsv_schedule(L, n, +1, group_of, ngroups, F, err) ||
                     !build_trsv_schedule(L, n, -1, group_of, ngroups, B, err))) {
    snprintf(msg, msglen, "%s", err.c_str());
    return -2;
  }
  // direct solves
  std::vector<double> y(n), z(n);
  for (int64_t i = 0; i < n; ++i) {
    double s = b[i];
    for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1] - 1; ++k) s -= Lval[k] * y[L.col[k]];
    y[i] = s / Lval[L.rowptr[i + 1] - 1];
  }
  std::vector<double> tmp(y);
  for (int64_t i = n - 1; i >= 0; --i) {
    const double zi = tmp[i] / Lval[L.rowptr[i + 1] - 1];
    z[i] = zi;
    for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1] - 1; ++k) tmp[L.col[k]] -= Lval[k] * zi;
  }
  Emu emu;
  long rf = 0, rb = 0;
  std::vector<double> yf = emulate(F, L, Lval, lrow, n, +1, b, emu, &rf);
  std::vector<double> zb;
  if (emu.ok) zb = emulate(B, L, Lval, lrow, n, -1, y, emu, &rb);
  double ef = 0, eb = 0;
  if (emu.ok)
    for (int64_t i = 0; i < n; ++i) {
      ef = std::max(ef, std::fabs(yf[i] - y[i]) / (std::fabs(y[i]) + 1e-300));
      eb = std::max(eb, std::fabs(zb[i] - z[i]) / (std::fabs(z[i]) + 1e-300));
    }
  stats[0] = F.nlevels;
  stats[1] = B.nlevels;
  stats[2] = F.ngroups;
  stats[3] = F.nsteps;
  stats[4] = B.nsteps;
  stats[5] = std::max(F.nslots, B.nslots);
  stats[6] = std::max(F.E, B.E);
  stats[7] = ef;
  stats[8] = eb;
  stats[9] = double(rf);
  stats[10] = double(rb);
  stats[11] = double(F.halo_row.size());
  stats[12] = std::max(F.max_deg, B.max_deg);
  stats[13] = double(F.ncpl);
  if (!emu.ok) {
    snprintf(msg, msglen, "%s", emu.msg);
    return -3;
  }
  return 0;
}

// Row ranges of the CSR row kernels for the saddle pattern (which = 0: all rows,
// 1: A part of the velocity rows) on num_cu CUs.  Call with null split to get nb.
int hc_row_split(int N, int kp, int dim, int which, int num_cu, int* nb, int32_t* split) {
  Spaces S = make_spaces(N, kp, dim);
  SaddlePattern P;
  std::string err;
  if (build_saddle_pattern(S, P, err) != 0) return -1;
  const int64_t nrows = which == 0 ? S.n_u + S.n_p : S.n_u;
  *nb = which == 0 ? row_split_blocks(nrows, num_cu) : row_split_blocks(nrows, num_cu, kPcgSpmvBlocksPerCU);
  if (split) {
    const std::vector<int32_t> v = balanced_row_split(P.rowptr, which == 0 ? nullptr : &P.aend, nrows, *nb);
    for (size_t i = 0; i < v.size(); ++i) split[i] = v[i];
  }
  return 0;
}

}  // extern "C"

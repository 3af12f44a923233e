// Host-side setup of libstokes.so: integer work only.
//  * discrete space sizes and the DOF numbering (Sec. 3.2 of the paper),
//  * the saddle-point CSR pattern in closed form (support overlap of tensor-product
//    B-splines, Sec. 2.2), the lower-triangle (IC(0)) pattern,
//  * dependency levels and the per-workgroup schedules of the triangular solves.
// No floating-point arithmetic of the method happens here: assembly, factorisation and
// all solver arithmetic run in the HIP kernels.
#include <algorithm>
#include <numeric>

#include "stokes_internal.h"

namespace stk {

Spaces make_spaces(int N, int kp, int dim) {
  Spaces S;
  S.N = N;
  S.kp = kp;
  S.dim = dim;
  S.pdeg = kp + 1;
  S.nlo = N + kp;
  S.nhi = N + kp + 1;
  int64_t off = 0;
  for (int c = 0; c < dim; ++c) {
    int64_t cnt = 1;
    for (int d = 0; d < dim; ++d) {
      if (d == c) {
        S.vcnt[c][d] = S.nhi - 2;  // first/last function of direction c removed (u.n = 0)
        S.vshift[c][d] = 1;
        S.vdeg[c][d] = S.pdeg;
      } else {
        S.vcnt[c][d] = S.nlo;
        S.vshift[c][d] = 0;
        S.vdeg[c][d] = kp;
      }
      cnt *= S.vcnt[c][d];
    }
    S.voff[c] = off;
    off += cnt;
  }
  S.voff[dim] = off;
  S.n_u = off;
  S.n_p = 1;
  for (int d = 0; d < dim; ++d) S.n_p *= S.nlo;
  return S;
}

namespace {

// 1D index range of functions (degree db, full index range [lo_valid, hi_valid]) whose
// support intersects the element range [elo, ehi]: b - db <= ehi and b >= elo.
inline void overlap_range(int elo, int ehi, int db, int lo_valid, int hi_valid, int* a, int* b) {
  *a = std::max(elo, lo_valid);
  *b = std::min(ehi + db, hi_valid);
}

struct RowDesc {
  int elo[3], ehi[3];  // element range of the row function's support per direction
};

// Append the sorted velocity columns (all components) and, if want_p, pressure columns
// overlapping the element box of `rd`.
template <typename Emit>
void emit_columns(const Spaces& S, const RowDesc& rd, bool want_p, Emit emit) {
  for (int d = 0; d < S.dim; ++d) {
    int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < S.dim; ++k) {
      int full_lo = S.vshift[d][k];
      int full_hi = S.vshift[d][k] + S.vcnt[d][k] - 1;
      overlap_range(rd.elo[k], rd.ehi[k], S.vdeg[d][k], full_lo, full_hi, &a[k], &b[k]);
    }
    int z0 = S.dim == 3 ? a[2] : 0, z1 = S.dim == 3 ? b[2] : 0;
    for (int z = z0; z <= z1; ++z)
      for (int y = a[1]; y <= b[1]; ++y) {
        int64_t base = S.voff[d];
        int64_t ly = y - S.vshift[d][1];
        int64_t lz = S.dim == 3 ? (z - S.vshift[d][2]) : 0;
        int64_t rowbase = base + (lz * S.vcnt[d][1] + ly) * S.vcnt[d][0];
        for (int x = a[0]; x <= b[0]; ++x) emit(rowbase + (x - S.vshift[d][0]));
      }
  }
  if (want_p) {
    int a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < S.dim; ++k) overlap_range(rd.elo[k], rd.ehi[k], S.kp, 0, S.nlo - 1, &a[k], &b[k]);
    int z0 = S.dim == 3 ? a[2] : 0, z1 = S.dim == 3 ? b[2] : 0;
    for (int z = z0; z <= z1; ++z)
      for (int y = a[1]; y <= b[1]; ++y) {
        int64_t rowbase = S.n_u + (int64_t(z) * S.nlo + y) * S.nlo;
        for (int x = a[0]; x <= b[0]; ++x) emit(rowbase + x);
      }
  }
}

void velocity_row_desc(const Spaces& S, int64_t g, int* comp, int* i1d, RowDesc& rd) {
  int c = 0;
  while (c + 1 < S.dim && g >= S.voff[c + 1]) ++c;
  int64_t r = g - S.voff[c];
  for (int d = 0; d < S.dim; ++d) {
    int i = int(r % S.vcnt[c][d]) + S.vshift[c][d];
    r /= S.vcnt[c][d];
    i1d[d] = i;
    rd.elo[d] = std::max(0, i - S.vdeg[c][d]);
    rd.ehi[d] = std::min(S.N - 1, i);
  }
  for (int d = S.dim; d < 3; ++d) rd.elo[d] = rd.ehi[d] = 0;
  *comp = c;
}

void pressure_row_desc(const Spaces& S, int64_t k, RowDesc& rd) {
  for (int d = 0; d < S.dim; ++d) {
    int i = int(k % S.nlo);
    k /= S.nlo;
    rd.elo[d] = std::max(0, i - S.kp);
    rd.ehi[d] = std::min(S.N - 1, i);
  }
  for (int d = S.dim; d < 3; ++d) rd.elo[d] = rd.ehi[d] = 0;
}

}  // namespace

int build_saddle_pattern(const Spaces& S, SaddlePattern& P, std::string& err) {
  const int64_t n = S.n_u + S.n_p;
  P.rowptr.assign(n + 1, 0);
  P.aend.assign(S.n_u, 0);
  // pass 1: counts
  int64_t total = 0;
  for (int64_t i = 0; i < n; ++i) {
    RowDesc rd;
    int c, i1d[3];
    int64_t cnt = 0, acnt = 0;
    if (i < S.n_u) {
      velocity_row_desc(S, i, &c, i1d, rd);
      emit_columns(S, rd, true, [&](int64_t j) {
        ++cnt;
        if (j < S.n_u) ++acnt;
      });
    } else {
      pressure_row_desc(S, i - S.n_u, rd);
      emit_columns(S, rd, false, [&](int64_t) { ++cnt; });
    }
    total += cnt;
    if (total >= (int64_t(1) << 31) - 1) {
      err = "saddle matrix has more than 2^31 non-zeros (int32 CSR)";
      return -1;
    }
    P.rowptr[i + 1] = int32_t(total);
    if (i < S.n_u) P.aend[i] = int32_t(P.rowptr[i] + acnt);
  }
  P.col.resize(total);
  for (int64_t i = 0; i < n; ++i) {
    RowDesc rd;
    int c, i1d[3];
    int64_t pos = P.rowptr[i];
    if (i < S.n_u) {
      velocity_row_desc(S, i, &c, i1d, rd);
      emit_columns(S, rd, true, [&](int64_t j) { P.col[pos++] = int32_t(j); });
    } else {
      pressure_row_desc(S, i - S.n_u, rd);
      emit_columns(S, rd, false, [&](int64_t j) { P.col[pos++] = int32_t(j); });
    }
  }
  return 0;
}

void build_lower_pattern(const Spaces& S, const SaddlePattern& P, LowerPattern& L) {
  L.rowptr.assign(S.n_u + 1, 0);
  L.col.clear();
  L.src.clear();
  for (int64_t i = 0; i < S.n_u; ++i) {
    for (int32_t k = P.rowptr[i]; k < P.aend[i]; ++k) {
      if (P.col[k] > i) break;
      L.col.push_back(P.col[k]);
      L.src.push_back(k);
    }
    L.rowptr[i + 1] = int32_t(L.col.size());
  }
}

void forward_levels(const LowerPattern& L, int64_t n, std::vector<int32_t>& lev, int* nlev) {
  lev.assign(n, 0);
  int mx = 0;
  for (int64_t i = 0; i < n; ++i) {
    int l = 0;
    for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1] - 1; ++k) l = std::max(l, lev[L.col[k]] + 1);
    lev[i] = l;
    mx = std::max(mx, l);
  }
  *nlev = mx + 1;
}

// Dependency lists of a triangular solve in processing order.  Forward, row i needs rows
// j < i of row i of L; backward, row i needs rows j > i with L_ji != 0 (column i of L below
// the diagonal).  dval holds the index of the coefficient in L's value array.
struct TrsvDeps {
  int64_t n = 0;                 // rows (with coupling rows: n_u + their number)
  std::vector<int64_t> dptr;     // [n+1]
  std::vector<int32_t> dcol;
  std::vector<int64_t> dval;
  std::vector<int64_t> diag;     // [n] index of the diagonal value
  std::vector<int32_t> order;    // [n] processing order
};

static void trsv_deps(const LowerPattern& L, int64_t n, int dir, TrsvDeps& D) {
  D.n = n;
  D.dptr.assign(n + 1, 0);
  D.dcol.clear();
  D.dval.clear();
  D.diag.resize(n);
  D.order.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    D.diag[i] = L.rowptr[i + 1] - 1;
    D.order[i] = int32_t(dir > 0 ? i : n - 1 - i);
  }
  if (dir > 0) {
    D.dcol.reserve(L.col.size());
    D.dval.reserve(L.col.size());
    for (int64_t i = 0; i < n; ++i) {
      for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1] - 1; ++k) {
        D.dcol.push_back(L.col[k]);
        D.dval.push_back(k);
      }
      D.dptr[i + 1] = int64_t(D.dcol.size());
    }
  } else {
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t k = L.rowptr[i]; k < L.rowptr[i + 1] - 1; ++k) cnt[L.col[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) D.dptr[i + 1] = D.dptr[i] + cnt[i + 1];
    D.dcol.resize(D.dptr[n]);
    D.dval.resize(D.dptr[n]);
    std::vector<int64_t> fill(D.dptr.begin(), D.dptr.end() - 1);
    for (int64_t j = 0; j < n; ++j)
      for (int32_t k = L.rowptr[j]; k < L.rowptr[j + 1] - 1; ++k) {
        const int64_t i = L.col[k];
        D.dcol[fill[i]] = int32_t(j);
        D.dval[fill[i]] = k;
        fill[i]++;
      }
  }
}

// Coupling rows.  The rows form consecutive blocks (blk: offsets, the velocity components),
// solved one after another; a row depends on rows of its own block and of blocks solved
// before it.  For each row i and each earlier block b it depends on, a coupling row
// c_ib = sum over those dependencies of the coefficient times the value is written as one
// more row of the triangular system (its dependencies with their coefficients, right-hand
// side 0, diagonal -1: (0 - sum)/(-1)), and row i keeps its own block's dependencies plus
// the c_ib with coefficient 1.  Processing order: each block, then the coupling rows whose
// dependencies lie in it.  cpl_row[k] and cpl_src[k] are the row and the block of coupling
// row n + k.
static void trsv_couple(TrsvDeps& D, const std::vector<int64_t>& blk, int dir, std::vector<int32_t>& cpl_row,
                        std::vector<int32_t>& cpl_src) {
  const int64_t n = D.n;
  const int nb = int(blk.size()) - 1;
  std::vector<int8_t> bof(n);
  for (int b = 0; b < nb; ++b)
    for (int64_t i = blk[b]; i < blk[b + 1]; ++i) bof[i] = int8_t(b);
  std::vector<int> border(nb);
  for (int b = 0; b < nb; ++b) border[b] = dir > 0 ? b : nb - 1 - b;
  // coupling rows numbered by source block in solve order, then by the dependent row's
  // processing position
  cpl_row.clear();
  cpl_src.clear();
  std::vector<int32_t> cidx(size_t(n) * nb, -1);
  for (int sb : border)
    for (int32_t i : D.order) {
      if (bof[i] == sb) continue;
      for (int64_t k = D.dptr[i]; k < D.dptr[i + 1]; ++k)
        if (bof[D.dcol[k]] == sb) {
          cidx[size_t(i) * nb + sb] = int32_t(n + int64_t(cpl_row.size()));
          cpl_row.push_back(i);
          cpl_src.push_back(sb);
          break;
        }
    }
  const int64_t nc = int64_t(cpl_row.size());
  TrsvDeps X;
  X.n = n + nc;
  X.dptr.assign(X.n + 1, 0);
  X.diag.resize(X.n);
  X.dcol.reserve(D.dcol.size() + nc);
  X.dval.reserve(D.dval.size() + nc);
  for (int64_t i = 0; i < n; ++i) {
    X.diag[i] = D.diag[i];
    for (int64_t k = D.dptr[i]; k < D.dptr[i + 1]; ++k)
      if (bof[D.dcol[k]] == bof[i]) {
        X.dcol.push_back(D.dcol[k]);
        X.dval.push_back(D.dval[k]);
      }
    for (int sb : border)
      if (cidx[size_t(i) * nb + sb] >= 0) {
        X.dcol.push_back(cidx[size_t(i) * nb + sb]);
        X.dval.push_back(kTrsvValOne);
      }
    X.dptr[i + 1] = int64_t(X.dcol.size());
  }
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t i = cpl_row[c];
    X.diag[n + c] = kTrsvValMinusOne;
    for (int64_t k = D.dptr[i]; k < D.dptr[i + 1]; ++k)
      if (bof[D.dcol[k]] == cpl_src[c]) {
        X.dcol.push_back(D.dcol[k]);
        X.dval.push_back(D.dval[k]);
      }
    X.dptr[n + c + 1] = int64_t(X.dcol.size());
  }
  X.order.clear();
  X.order.reserve(X.n);
  int64_t c = 0;
  for (int sb : border) {
    for (int32_t i : D.order)
      if (bof[i] == sb) X.order.push_back(i);
    for (; c < nc && cpl_src[c] == sb; ++c) X.order.push_back(int32_t(n + c));
  }
  D = std::move(X);
}

static std::vector<int32_t> trsv_levels(const TrsvDeps& D, int* nlevels) {
  std::vector<int32_t> lev(D.n, 0);
  int maxlev = 0;
  for (int32_t i : D.order) {
    int l = 0;
    for (int64_t k = D.dptr[i]; k < D.dptr[i + 1]; ++k) l = std::max(l, lev[D.dcol[k]] + 1);
    lev[i] = l;
    maxlev = std::max(maxlev, l);
  }
  *nlevels = maxlev + 1;
  return lev;
}

static bool schedule_core(const TrsvDeps& D, const std::vector<int32_t>& lev, int nlevels,
                          const std::vector<int32_t>& group_of, int ngroups, const std::vector<char>& pack,
                          TrsvSchedHost& S, std::string& err);

bool build_trsv_schedule(const LowerPattern& L, int64_t n, int dir, const std::vector<int32_t>& group_of,
                         int ngroups, TrsvSchedHost& S, std::string& err) {
  TrsvDeps D;
  trsv_deps(L, n, dir, D);
  int nl = 0;
  const std::vector<int32_t> lev = trsv_levels(D, &nl);
  S.nrows = n;
  S.ncpl = 0;
  S.cpl_row.clear();
  S.grp_cpl.assign(ngroups, 0);
  return schedule_core(D, lev, nl, group_of, ngroups, std::vector<char>(ngroups, 0), S, err);
}

bool build_trsv_schedule_coupled(const LowerPattern& L, int64_t n, int dir, const std::vector<int64_t>& blk,
                                 int helpers, const std::vector<int32_t>& group_of, int ngroups, TrsvSchedHost& S,
                                 std::string& err) {
  TrsvDeps D;
  trsv_deps(L, n, dir, D);
  std::vector<int32_t> cpl_row, cpl_src;
  trsv_couple(D, blk, dir, cpl_row, cpl_src);
  int nl = 0;
  const std::vector<int32_t> lev = trsv_levels(D, &nl);
  const int64_t nc = int64_t(cpl_row.size());
  const int nb = int(blk.size()) - 1;
  // helper groups: `helpers` per (group of the dependent row, source block); the coupling
  // rows of one such pair in (level, processing) order are dealt to its helpers in runs of
  // one step
  std::vector<int32_t> hbase(size_t(ngroups) * nb, -1);
  int ng = ngroups;
  for (int64_t c = 0; c < nc; ++c) {
    const size_t key = size_t(group_of[cpl_row[c]]) * nb + cpl_src[c];
    if (hbase[key] < 0) {
      hbase[key] = ng;
      ng += helpers;
    }
  }
  std::vector<int32_t> gx(group_of);
  gx.resize(D.n, 0);
  std::vector<std::vector<int32_t>> per(size_t(ngroups) * nb);
  for (int32_t i : D.order)
    if (i >= n) per[size_t(group_of[cpl_row[i - n]]) * nb + cpl_src[i - n]].push_back(i);
  for (size_t key = 0; key < per.size(); ++key) {
    auto& v = per[key];
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return lev[a] < lev[b]; });
    for (size_t r = 0; r < v.size(); ++r) gx[v[r]] = hbase[key] + int32_t((r / kTrsvRPS) % helpers);
  }
  std::vector<char> pack(ng, 0);
  for (int g = ngroups; g < ng; ++g) pack[g] = 1;
  S.nrows = n;
  S.ncpl = nc;
  S.cpl_row = cpl_row;
  S.grp_cpl.assign(ng, 0);
  for (int g = ngroups; g < ng; ++g) S.grp_cpl[g] = 1;
  return schedule_core(D, lev, nl, gx, ng, pack, S, err);
}

// Steps, LDS slots and halo lists of a schedule.  A group's rows are taken in (level,
// processing) order, in steps of <= kTrsvRPS rows of one level; a packed group (whose rows
// do not depend on each other) fills every step regardless of level.
static bool schedule_core(const TrsvDeps& D, const std::vector<int32_t>& lev, int nlevels,
                          const std::vector<int32_t>& group_of, int ngroups, const std::vector<char>& pack,
                          TrsvSchedHost& S, std::string& err) {
  const int64_t n = D.n;
  const std::vector<int64_t>& dptr = D.dptr;
  const std::vector<int32_t>& dcol = D.dcol;
  const std::vector<int64_t>& dval = D.dval;
  const std::vector<int64_t>& diag = D.diag;
  S.nlevels = nlevels;
  int maxdeg = 0;
  for (int64_t i = 0; i < n; ++i) maxdeg = std::max<int>(maxdeg, int(dptr[i + 1] - dptr[i]));
  S.max_deg = maxdeg;
  S.E = std::max(1, (maxdeg + kTrsvG - 1) / kTrsvG);
  if (S.E > 16) {
    err = "triangular-solve rows have more than 16*G dependencies";
    return false;
  }
  S.ngroups = ngroups;
  const int RPS = kTrsvRPS, E = S.E;

  // rows of each group sorted by (level, processing order); steps of <= RPS rows of one level
  std::vector<std::vector<int32_t>> grows(ngroups);
  for (int32_t i : D.order) grows[group_of[i]].push_back(i);
  std::vector<int32_t> step_of(n, -1);  // group-relative step of each row
  std::vector<std::vector<int32_t>> gstep_begin(ngroups);  // row offsets of steps in grows[g]
  for (int g = 0; g < ngroups; ++g) {
    auto& v = grows[g];
    std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return lev[a] < lev[b]; });
    auto& sb = gstep_begin[g];
    size_t k = 0;
    while (k < v.size()) {
      const int lv = lev[v[k]];
      size_t k1 = k;
      while (k1 < v.size() && (pack[g] || lev[v[k1]] == lv) && int(k1 - k) < RPS) ++k1;
      for (size_t r = k; r < k1; ++r) step_of[v[r]] = int32_t(sb.size());
      sb.push_back(int32_t(k));
      k = k1;
    }
    sb.push_back(int32_t(v.size()));
  }
  // requested publish levels: (producer group, level) of every remote dependency
  std::vector<std::vector<int32_t>> pub_levels(ngroups);
  S.grp_step_ptr.assign(ngroups + 1, 0);
  S.grp_halo_ptr.assign(ngroups + 1, 0);
  S.halo_row.clear();
  S.halo_grp.clear();
  S.halo_lvl.clear();
  S.halo_slot.clear();
  S.halo_free.clear();
  S.step_level.clear();
  S.step_halo_need.clear();
  S.step_publish.clear();
  S.srow.clear();
  S.sslot.clear();
  S.sdiag_src.clear();
  S.ent_src.clear();
  S.ent_perm.clear();
  S.ent_dep.clear();
  S.nslots = 1;

  struct HaloTmp {
    int32_t row, first, last;
  };
  std::vector<int32_t> slot_of(n, 0);
  std::vector<int32_t> last_local(n, -1);
  int nsteps_total = 0;
  for (int g = 0; g < ngroups; ++g) {
    const auto& v = grows[g];
    const auto& sb = gstep_begin[g];
    const int ns = int(sb.size()) - 1;
    // local last use and halo first/last use
    std::vector<HaloTmp> halo;
    {
      std::vector<std::pair<int32_t, int32_t>> uses;  // (remote row, step)
      for (int32_t i : v)
        for (int64_t k = dptr[i]; k < dptr[i + 1]; ++k) {
          const int32_t j = dcol[k];
          if (group_of[j] == g) {
            last_local[j] = std::max(last_local[j], step_of[i]);
          } else {
            uses.push_back({j, step_of[i]});
          }
        }
      std::sort(uses.begin(), uses.end());
      for (size_t a = 0; a < uses.size();) {
        size_t b = a;
        int32_t f = uses[a].second, l = uses[a].second;
        while (b < uses.size() && uses[b].first == uses[a].first) {
          f = std::min(f, uses[b].second);
          l = std::max(l, uses[b].second);
          ++b;
        }
        halo.push_back({uses[a].first, f, l});
        a = b;
      }
      std::stable_sort(halo.begin(), halo.end(), [&](const HaloTmp& x, const HaloTmp& y) {
        if (x.first != y.first) return x.first < y.first;
        if (lev[x.row] != lev[y.row]) return lev[x.row] < lev[y.row];
        return x.row < y.row;
      });
    }
    // interval slot allocation over steps
    std::vector<int32_t> halo_slot(halo.size(), 0), halo_free(halo.size(), 0);
    {
      std::vector<int32_t> free_slots;          // stack
      std::vector<int32_t> slot_end_prev;       // last use (step) of the previous occupant per slot
      slot_end_prev.push_back(-1);              // slot 0 (zero slot) never allocated
      // release lists: slots to free after step k
      std::vector<std::vector<int32_t>> release(ns + 1);
      auto alloc = [&](int32_t end, int32_t* prev_end) {
        int32_t s;
        if (!free_slots.empty()) {
          s = free_slots.back();
          free_slots.pop_back();
        } else {
          s = int32_t(slot_end_prev.size());
          slot_end_prev.push_back(-1);
        }
        *prev_end = slot_end_prev[s];
        slot_end_prev[s] = end;
        release[std::min(end, ns - 1) + 1].push_back(s);
        return s;
      };
      size_t hpos = 0;
      for (int k = 0; k < ns; ++k) {
        for (int32_t s : release[k]) free_slots.push_back(s);
        // halo entries whose window starts at step k
        while (hpos < halo.size() && std::max(0, halo[hpos].first - kTrsvHaloLookahead) <= k) {
          int32_t pe;
          halo_slot[hpos] = alloc(halo[hpos].last, &pe);
          halo_free[hpos] = pe + 1;  // the previous occupant's last use must be computed
          ++hpos;
        }
        // local rows computed at step k that have local consumers
        for (int32_t r = sb[k]; r < sb[k + 1]; ++r) {
          const int32_t i = v[r];
          if (last_local[i] >= 0) {
            int32_t pe;
            slot_of[i] = alloc(last_local[i], &pe);
          } else {
            slot_of[i] = 0;
          }
        }
      }
      S.nslots = std::max<int>(S.nslots, int(slot_end_prev.size()));
    }
    // halo records (and publish requests)
    for (size_t h = 0; h < halo.size(); ++h) {
      const int32_t j = halo[h].row;
      S.halo_row.push_back(j);
      S.halo_grp.push_back(group_of[j]);
      S.halo_lvl.push_back(lev[j]);
      S.halo_slot.push_back(halo_slot[h]);
      S.halo_free.push_back(halo_free[h]);
      pub_levels[group_of[j]].push_back(lev[j]);
    }
    S.grp_halo_ptr[g + 1] = int32_t(S.halo_row.size());
    // slot lookup for halo rows of this group
    std::vector<std::pair<int32_t, int32_t>> hidx(halo.size());
    for (size_t h = 0; h < halo.size(); ++h) hidx[h] = {halo[h].row, halo_slot[h]};
    std::sort(hidx.begin(), hidx.end());
    // steps
    size_t hneed = 0;
    for (int k = 0; k < ns; ++k) {
      while (hneed < halo.size() && halo[hneed].first <= k) ++hneed;
      const size_t base_sr = S.srow.size(), base_e = S.ent_src.size();
      S.srow.resize(base_sr + RPS, -1);
      S.sslot.resize(base_sr + RPS, 0);
      S.sdiag_src.resize(base_sr + RPS, -1);
      S.ent_src.resize(base_e + size_t(E) * 64, 0);
      S.ent_perm.resize(base_e + size_t(E) * 64, -1);
      S.ent_dep.resize(base_e + size_t(E) * 64, -1);
      for (int32_t r = sb[k]; r < sb[k + 1]; ++r) {
        const int32_t i = v[r];
        const int rr = r - sb[k];
        S.srow[base_sr + rr] = i;
        S.sslot[base_sr + rr] = slot_of[i];
        S.sdiag_src[base_sr + rr] = diag[i];
        int m = 0;
        for (int64_t q = dptr[i]; q < dptr[i + 1]; ++q, ++m) {
          const int32_t j = dcol[q];
          const int lane = rr * kTrsvG + (m % kTrsvG);
          const int e = m / kTrsvG;
          int32_t src;
          if (group_of[j] == g) {
            src = slot_of[j];
          } else {
            auto it = std::lower_bound(hidx.begin(), hidx.end(), std::make_pair(j, int32_t(-1)));
            src = it->second;
          }
          S.ent_src[base_e + size_t(e) * 64 + lane] = src;
          S.ent_perm[base_e + size_t(e) * 64 + lane] = dval[q];
          S.ent_dep[base_e + size_t(e) * 64 + lane] = j;
        }
      }
      S.step_level.push_back(lev[v[sb[k]]]);
      S.step_halo_need.push_back(int32_t(hneed));
      S.step_publish.push_back(0);
    }
    nsteps_total += ns;
    S.grp_step_ptr[g + 1] = nsteps_total;
  }
  S.nsteps = nsteps_total;
  // publish after the last step of every requested level
  for (int g = 0; g < ngroups; ++g) {
    auto& pl = pub_levels[g];
    std::sort(pl.begin(), pl.end());
    pl.erase(std::unique(pl.begin(), pl.end()), pl.end());
    for (int k = S.grp_step_ptr[g]; k < S.grp_step_ptr[g + 1]; ++k) {
      const bool last_of_level = (k + 1 == S.grp_step_ptr[g + 1]) || S.step_level[k + 1] != S.step_level[k];
      if (last_of_level && std::binary_search(pl.begin(), pl.end(), S.step_level[k])) S.step_publish[k] = 1;
    }
  }
  (void)err;
  return true;
}

// Strip partition: rows of velocity component c with last-direction 1D index t belong to
// group offset_c + t / strip.
void strip_groups(const Spaces& S, int strip, std::vector<int32_t>& group_of, int* ngroups) {
  group_of.assign(S.n_u, 0);
  int off = 0;
  const int last = S.dim - 1;
  for (int c = 0; c < S.dim; ++c) {
    int64_t inner = 1;
    for (int d = 0; d < last; ++d) inner *= S.vcnt[c][d];
    const int nt = S.vcnt[c][last];
    const int ns = (nt + strip - 1) / strip;
    for (int64_t k = 0; k < S.voff[c + 1] - S.voff[c]; ++k) {
      const int t = int(k / inner);
      group_of[S.voff[c] + k] = off + t / strip;
    }
    off += ns;
  }
  *ngroups = off;
}

}  // namespace stk

// ---------------------------------------------------------------------------
// Row ranges for the CSR row kernels, balanced by work: a row costs its entries plus a
// fixed amount for the per-row loads and stores (kRowCost entries' worth).
// ---------------------------------------------------------------------------
namespace stk {

int row_split_blocks(int64_t nrows, int num_cu, int per_cu) {
  const int64_t cap = (int64_t)std::max(1, per_cu) * std::max(1, num_cu);
  int64_t nb = std::max<int64_t>(1, std::min<int64_t>(cap, (nrows + 15) / 16));
  nb = std::min<int64_t>(nb, kVecMaxBlocks);
  if (nb > 8) nb = nb / 8 * 8;
  return (int)nb;
}

std::vector<int32_t> balanced_row_split(const std::vector<int32_t>& rowptr, const std::vector<int32_t>* rowend,
                                        int64_t nrows, int nb) {
  constexpr int64_t kRowCost = 16;
  auto len = [&](int64_t i) -> int64_t { return (rowend ? (*rowend)[i] : rowptr[i + 1]) - rowptr[i]; };
  int64_t total = 0;
  for (int64_t i = 0; i < nrows; ++i) total += len(i) + kRowCost;
  std::vector<int32_t> split(nb + 1, 0);
  int64_t i = 0, acc = 0;
  for (int b = 1; b < nb; ++b) {
    const int64_t target = (total * b) / nb;
    while (i < nrows && acc + len(i) + kRowCost <= target) {
      acc += len(i) + kRowCost;
      ++i;
    }
    split[b] = (int32_t)i;
  }
  split[nb] = (int32_t)nrows;
  return split;
}

}  // namespace stk

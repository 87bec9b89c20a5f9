// Host runtime of libamg: gauge handles, the multigrid hierarchy, setup
// (given or adaptive near-null vectors), the V-cycle, FGCR and CGNR, and the
// C ABI declared in include/amg.h.  Every arithmetic step runs in the gfx950
// kernels of this library; the host only sequences launches and reads one
// residual norm per outer iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "amg.h"
#include "kernels.h"
#include "dispatch.h"
#include "hostutil.h"
#include "gauge.h"

using namespace amg;
using namespace amg::host;

namespace amg {
namespace host {
std::string& last_error() {
  thread_local std::string msg;
  return msg;
}
}  // namespace host
}  // namespace amg

namespace amg {
Recorder*& current_recorder() {
  thread_local Recorder* rec = nullptr;
  return rec;
}
LaunchTiming& pending_timing() {
  thread_local LaunchTiming t;
  return t;
}
namespace {
thread_local int g_red_cap = RED_MAX_BLOCKS;
}
int red_block_cap() { return g_red_cap; }
void set_red_block_cap(int cap) { g_red_cap = std::max(16, std::min(RED_MAX_BLOCKS, cap)); }
}  // namespace amg

namespace {

template <typename T> struct Pick;
template <> struct Pick<double> { static constexpr int prec = AMG_F64; };
template <> struct Pick<float> { static constexpr int prec = AMG_F32; };

// slots of one GCR instance in the scalar array
struct GcrSlots {
  int beta, ww, alpha, rr, bb;
  static int size() { return RHS_MAX * GCR_KMAX * 3 + RHS_MAX * 4; }
  void at(int base) {
    beta = base;
    ww = beta + RHS_MAX * GCR_KMAX * 2;
    alpha = ww + RHS_MAX * GCR_KMAX;
    rr = alpha + RHS_MAX * 2;
    bb = rr + RHS_MAX;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// multigrid hierarchy
// ---------------------------------------------------------------------------
namespace {

enum { W_B = 0, W_X, W_R, W_P, W_GR, W_COUNT };

struct Level {
  bool fine = false;
  int nd = 2;
  int dims[4] = {1, 1, 1, 1};
  long V = 0;
  int dof = 0;       // current dof per site
  int dof_max = 0;   // allocation size (coarse levels grow during adaptive setup)
  Layout lay64, lay32;
  // coarse operator (levels >= 1): Y [V][2nd+1][dof][dof], mass matrix M [V][dof][dof]
  Buf Y64, Y32, M64;
  // transfer to the next level
  bool has_next = false;
  int blk[4] = {1, 1, 1, 1};
  int nv = 0, nv_max = 0;
  Buf vecs;          // raw near-null vectors [nv][per_rhs] (lay64)
  Buf P64, P32, Pbf; // [Vc][bs][dof][nv]
  // work vectors (per precision)
  Buf w64[W_COUNT], w32[W_COUNT];
  Buf Z64, W64, Z32, W32;  // GCR directions (coarsest level)
  // exact coarsest solve: dense inverse of this level's operator (FP64, and
  // FP32 for the FP32 cycle), valid while `dense` is set
  Buf D64, D32;
  bool dense = false;
  // right block-Jacobi preconditioning of this level's GCR as the coarsest
  // level: M = inverse diagonal blocks, J = the stencil of A M (both FP64,
  // and FP32 for the FP32 cycle), JY = the GCR iterate y (x = M y); valid
  // while `jac` is set
  Buf MI64, MI32, J64, J32, JY64, JY32;
  bool jac = false;
  // even-odd reduction of A M (2d levels with even extents): coupling blocks
  // of the even and the odd sites, scratch for T_oe z and the reduced
  // right-hand side; valid while `eo` is set
  Buf CE64, CO64, CE32, CO32, EO64, EO32;
  bool eo = false;
  // with 16 dof also the reduced operator as a 9-point stencil of the even
  // sites (one launch per product instead of two)
  Buf SE64, SE32;
  bool s9 = false;
  int alloc_nrhs = 0;
  // scalar slots
  int mr_slot = 0;
  GcrSlots gs;
  int flag_off = 0;

  long per_rhs() const { return V * dof; }
  int ndir() const { return 2 * nd + 1; }
  CoarseGeom cgeom() const {
    CoarseGeom c;
    c.nd = nd;
    for (int i = 0; i < 4; ++i) c.dims[i] = dims[i];
    c.V = V;
    c.nc = dof;
    return c;
  }
  template <typename T> Buf* w() { return Pick<T>::prec == AMG_F64 ? w64 : w32; }
  template <typename T> Buf& Zd() { return Pick<T>::prec == AMG_F64 ? Z64 : Z32; }
  template <typename T> Buf& Wd() { return Pick<T>::prec == AMG_F64 ? W64 : W32; }
  template <typename T> Layout lay() const { return Pick<T>::prec == AMG_F64 ? lay64 : lay32; }
  template <typename T> const cplx<T>* Y() const;
};
template <> const double2* Level::Y<double>() const { return Y64.as<double2>(); }
template <> const float2* Level::Y<float>() const { return Y32.as<float2>(); }
template <typename T> const cplx<T>* level_J(const Level& L) {
  return reinterpret_cast<const cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.J64.p : L.J32.p);
}
template <typename T> const cplx<T>* level_MI(const Level& L) {
  return reinterpret_cast<const cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.MI64.p : L.MI32.p);
}
template <typename T> cplx<T>* level_JY(Level& L) {
  return reinterpret_cast<cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.JY64.p : L.JY32.p);
}
template <typename T> const cplx<T>* level_CE(const Level& L) {
  return reinterpret_cast<const cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.CE64.p : L.CE32.p);
}
template <typename T> const cplx<T>* level_CO(const Level& L) {
  return reinterpret_cast<const cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.CO64.p : L.CO32.p);
}
template <typename T> const cplx<T>* level_SE(const Level& L) {
  return reinterpret_cast<const cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.SE64.p : L.SE32.p);
}
template <typename T> cplx<T>* level_EO(Level& L) {
  return reinterpret_cast<cplx<T>*>(Pick<T>::prec == AMG_F64 ? L.EO64.p : L.EO32.p);
}

}  // namespace

struct amg_solver {
  const amg_gauge* g = nullptr;
  amg_mg_params p;
  double mass = 0.0;
  std::vector<Level> lv;
  Scratch sc;
  int flags_base = 0;
  // outer FGCR (fine FP64)
  Buf ox, orr, ob, oZ, oW, otmp;
  int o_nrhs = 0;
  int outer_slot = 0;
  GcrSlots og;
  // setup temporaries
  Buf tE, tF, tS, tR, tzero;
  // Gauss-Jordan work (two N x N matrices, pivot records)
  Buf gjA, gjB, gjkey, gjint;
  Buf jerr;  // singular-block flag of the block-Jacobi set-up
  // batched solves run the coarsest level by GCR on every instance (one
  // launch sequence for all of them)
  bool no_dense = false;
  long long nD = 0, nDd = 0, nC = 0;
  // per-rhs mask of right-hand sides that are done (batched solves); nullptr otherwise
  int* outer_flags = nullptr;
  // persistent coarsest solve: barrier counters, timeout flag, iteration counts
  Buf pbar, perr, piters;
  bool persistent = false;  // measured slower than the launch sequence (grid barriers are costly)
  int pcoarse_max_blocks = 64;
  bool pcoarse_coop = true;
  bool fused_gcr = false;  // measured slower than the separate kernels at the 2d coarse sizes
  // GCR step as apply + one reduction for the orthogonalisation + update
  // (three launches) instead of apply + dots + orthogonalise + update
  bool gcr_dots = true;
  // FP32 coarse applies with at least this many right-hand sides use the
  // MFMA multi-rhs kernel (plain / residual epilogues, N_c = 16 or 48)
  int mrhs_min = 2;
  // kernel timing
  struct Prof {
    bool on = false;
    int kind = -1, level = -1;   // -1: every kind / every level
    std::vector<hipEvent_t> ev;  // start/stop pairs, reused
    std::vector<int> tag;        // (kind << 8 | level) of each pair
    size_t used = 0;
    hipStream_t last = nullptr;
  } prof;
  ~amg_solver() {
    for (auto e : prof.ev) (void)hipEventDestroy(e);
  }
};

namespace {

using Solver = amg_solver;

enum { PK_FINE = 0, PK_COARSE = 1, PK_RESTRICT = 2, PK_PROLONG = 3, PK_COARSE_MR = 4, PK_EO = 5, PK_EO_S9 = 6 };

// event pair around one launch when the profiler watches (kind, level)
struct ProfScope {
  Solver& S;
  bool active;
  hipStream_t st;
  ProfScope(Solver& s, int kind, int level, hipStream_t stream)
      : S(s),
        active(s.prof.on && (s.prof.kind == kind || s.prof.kind < 0) && (s.prof.level == level || s.prof.level < 0) &&
               current_recorder() == nullptr),
        st(stream) {
    if (!active) return;
    auto& P = S.prof;
    while (P.ev.size() < P.used + 2) {
      hipEvent_t e;
      HIPC(hipEventCreate(&e));
      P.ev.push_back(e);
    }
    if (P.tag.size() < P.used / 2 + 1) P.tag.resize(P.used / 2 + 1);
    P.tag[P.used / 2] = (kind << 8) | level;
    // the scope's (first) kernel launch stamps the pair
    pending_timing() = LaunchTiming{P.ev[P.used], P.ev[P.used + 1]};
  }
  ~ProfScope() {
    if (!active) return;
    auto& P = S.prof;
    LaunchTiming& t = pending_timing();
    if (t.start != nullptr) {  // nothing was launched: an empty interval
      (void)hipEventRecord(t.start, st);
      (void)hipEventRecord(t.stop, st);
      t = LaunchTiming{};
    }
    P.used += 2;
    P.last = st;
  }
};

TransferGeom tgeom(const Solver& S, int l, int prec) {
  const Level& f = S.lv[l];
  const Level& c = S.lv[l + 1];
  TransferGeom g;
  g.nd = f.nd;
  g.bs = 1;
  for (int mu = 0; mu < 4; ++mu) {
    g.fdims[mu] = f.dims[mu];
    g.blk[mu] = f.blk[mu];
    g.cdims[mu] = c.dims[mu];
    if (mu < f.nd) g.bs *= f.blk[mu];
  }
  g.Vf = f.V;
  g.Vc = c.V;
  g.dof = f.dof;
  g.nv = f.nv;
  g.lf = prec == AMG_F64 ? f.lay64 : f.lay32;
  return g;
}

template <typename T>
const void* Pstore(const Solver& S, int l, int& kind) {
  const Level& L = S.lv[l];
  if (Pick<T>::prec == AMG_F64) { kind = P_F64; return L.P64.p; }
  if (S.p.p_bf16) { kind = P_BF16; return L.Pbf.p; }
  kind = P_F32;
  return L.P32.p;
}

// operator of level l, precision T
template <typename T>
void op_apply(Solver& S, int l, int dagger, int epi, const cplx<T>* in, cplx<T>* out, const cplx<T>* b,
              cplx<T>* copy_out, int nrhs, RedArgs red, hipStream_t st, const cplx<T>* Yop = nullptr) {
  Level& L = S.lv[l];
  const bool mr_epi = epi == EPI_MRDOT || epi == EPI_MRPART;
  ProfScope ps(S, L.fine ? PK_FINE : (mr_epi && (S.prof.kind == PK_COARSE_MR || S.prof.kind < 0) ? PK_COARSE_MR
                                                                                                   : PK_COARSE),
               l, st);
  if (L.fine) {
    wilson_apply<T>(*S.g, S.mass, dagger, epi, in, out, b, copy_out, nrhs, red, st);
    (dagger ? S.nDd : S.nD) += 1;
  } else {
    CoarseArgs<T> a;
    a.out = out; a.in = in; a.b = b; a.copy_out = copy_out;
    a.Y = Yop ? Yop : L.Y<T>();
    a.g = L.cgeom();
    a.nrhs = nrhs;
    a.red = red;
    if (std::is_same<T, float>::value && nrhs >= S.mrhs_min && coarse_mrhs_supported(L.dof, epi))
      launch_coarse_mrhs(reinterpret_cast<const CoarseArgs<float>&>(a), dagger, epi, st);
    else
      launch_coarse<T>(a, dagger, epi, st);
    S.nC += 1;
  }
}

void alloc_level_work(Level& L, int nrhs, int restart, bool coarsest, bool f32) {
  if (L.alloc_nrhs >= nrhs) return;
  const size_t n = (size_t)L.V * L.dof_max * nrhs;
  for (int i = 0; i < W_COUNT; ++i) {
    L.w64[i].ensure(n * sizeof(double2));
    if (f32) L.w32[i].ensure(n * sizeof(float2));
  }
  if (coarsest) {
    L.Z64.ensure(n * restart * sizeof(double2));
    L.W64.ensure(n * restart * sizeof(double2));
    L.JY64.ensure(n * sizeof(double2));
    L.EO64.ensure(n * sizeof(double2));
    if (f32) {
      L.JY32.ensure(n * sizeof(float2));
      L.EO32.ensure(n * sizeof(float2));
    }
    if (f32) {
      L.Z32.ensure(n * restart * sizeof(float2));
      L.W32.ensure(n * restart * sizeof(float2));
    }
  }
  L.alloc_nrhs = nrhs;
}

void ensure_work(Solver& S, int nrhs) {
  if (nrhs > RHS_MAX) fail(AMG_ERR_ARG, "nrhs exceeds " + std::to_string(RHS_MAX));
  const bool f32 = S.p.inner_prec == AMG_F32;
  const int nl = (int)S.lv.size();
  for (int l = 0; l < nl; ++l) {
    // during adaptive setup every level may serve as the coarsest one
    alloc_level_work(S.lv[l], nrhs, std::max(S.p.coarse_restart, S.p.kcycle_maxiter), l > 0, f32);
  }
  if (S.o_nrhs < nrhs) {
    const size_t n = (size_t)S.lv[0].V * S.lv[0].dof * nrhs;
    S.ox.ensure(n * sizeof(double2));
    S.orr.ensure(n * sizeof(double2));
    S.ob.ensure(n * sizeof(double2));
    S.otmp.ensure(n * sizeof(double2));
    S.oZ.ensure(n * S.p.outer_restart * sizeof(double2));
    S.oW.ensure(n * S.p.outer_restart * sizeof(double2));
    S.o_nrhs = nrhs;
  }
}

// ---- smoother ---------------------------------------------------------------
// first = true:  x = MR_nu(b) from x = 0, r its residual;
// first = false: b is the current residual (may alias r), x += MR_nu(b).
template <typename T>
void mr_smooth(Solver& S, int l, const cplx<T>* b, cplx<T>* x, cplx<T>* r, cplx<T>* p, int nu, bool first,
               bool need_r, int nrhs, hipStream_t st) {
  Level& L = S.lv[l];
  const long n = L.per_rhs();
  if (nu == 0) {
    if (first) {
      launch_fill<T>(x, nullptr, n, nrhs, st);
      if (need_r && r != b) launch_fill<T>(r, b, n, nrhs, st);
    }
    return;
  }
  // N_c = 16 coarse levels: the stencil leaves per-block sums and the update
  // kernel forms alpha from them (no cross-block reduction in the stencil).
  // Not while recording for a batch: merged launches change the stencil's
  // grid, which the update kernel must know.
  const bool part = !L.fine && L.dof == 16 && current_recorder() == nullptr &&
                    coarse16_red_blocks(L.V) <= RED_MAX_PART_BLOCKS;
  for (int i = 0; i < nu; ++i) {
    const cplx<T>* rin = (i == 0) ? b : r;
    const bool upd = (i < nu - 1) || need_r;
    if (part) {
      op_apply<T>(S, l, 0, EPI_MRPART, rin, p, nullptr, nullptr, nrhs, S.sc.red(0, S.outer_flags), st);
      launch_mr_update<T>(x, r, rin, p, nullptr, n, nrhs, first && i == 0, upd ? 1 : 0, S.outer_flags, st,
                          S.sc.part.as<double>(), coarse16_red_blocks(L.V), S.p.omega);
      continue;
    }
    op_apply<T>(S, l, 0, EPI_MRDOT, rin, p, nullptr, nullptr, nrhs, S.sc.red(L.mr_slot, S.outer_flags, S.p.omega), st);
    launch_mr_update<T>(x, r, rin, p, S.sc.scal.as<double>() + L.mr_slot, n, nrhs, first && i == 0, upd ? 1 : 0,
                        S.outer_flags, st);
  }
}

constexpr int kCoarseCheck = 8;  // unpreconditioned GCR iterations between flag checks

template <typename T>
void vcycle(Solver& S, int l, int lstop, const cplx<T>* b, cplx<T>* x, int nrhs, hipStream_t st);

// ---- coarsest level, even-odd reduced: T = A M (block Jacobi, unit
// diagonal) split by parity; GCR on (1 - T_eo T_oe) y_e = b_e - T_eo b_o in
// the three-launch form of level_gcr (the product with the reduced operator
// is one 9-point stencil launch with 16 dof, else two half-lattice hops),
// then y_o = b_o - T_oe y_e and x = M y.  Stopping test |r_e| <= tol |b| on
// the full right-hand side: the odd residual is zero.
template <typename T>
void eo_gcr(Solver& S, int l, const cplx<T>* b, cplx<T>* x_out, int nrhs, double tol, int maxiter, int m,
            hipStream_t st) {
  Level& L = S.lv[l];
  const int L1 = L.dims[0], L2 = L.dims[1], nc = L.dof;
  const long n = L.per_rhs(), nh = n / 2;
  const long dstride = nh * nrhs;
  cplx<T>* ye = level_JY<T>(L);
  cplx<T>* yo = ye + dstride;
  cplx<T>* tmp = level_EO<T>(L);
  cplx<T>* bp = tmp + dstride;
  const cplx<T>* Ce = level_CE<T>(L);
  const cplx<T>* Co = level_CO<T>(L);
  Buf* w = L.w<T>();
  cplx<T>* r = w[W_GR].as<cplx<T>>();
  cplx<T>* Zb = L.template Zd<T>().template as<cplx<T>>();
  cplx<T>* Wb = L.template Wd<T>().template as<cplx<T>>();
  int* flags = S.sc.flags.as<int>() + L.flag_off;
  const double tol2 = tol * tol;
  // out = S v (epi 1) or bb - S v (epi 2), S = 1 - T_eo T_oe
  auto schur = [&](const cplx<T>* v, cplx<T>* out, const cplx<T>* bb, int epi) {
    if (L.s9) {
      ProfScope ps(S, PK_EO_S9, l, st);
      launch_eo_s9<T>(out, v, bb, level_SE<T>(L), L1, L2, epi == 2 ? 1 : 0, nrhs, st);
      S.nC += 1;
      return;
    }
    {
      ProfScope ps(S, PK_EO, l, st);
      launch_eo_hop<T>(tmp, v, nullptr, nullptr, Co, L1, L2, nc, 1, 0, 0, 0, nrhs, st);  // T_oe v
    }
    {
      ProfScope ps(S, PK_EO, l, st);
      launch_eo_hop<T>(out, tmp, bb, v, Ce, L1, L2, nc, 0, 0, 0, epi, nrhs, st);
    }
    S.nC += 1;
  };
  {
    // b' = b_e - T_eo b_o, also into r; y_e = 0
    ProfScope ps(S, PK_EO, l, st);
    launch_eo_hop<T>(bp, b, b, nullptr, Ce, L1, L2, nc, 0, 1, 1, 1, nrhs, st, r, ye);
  }
  launch_norm2<T>(b, n, nrhs, S.sc.red(L.gs.bb), st);
  launch_set_flags(flags, S.outer_flags, S.sc.scal.as<double>(), L.gs.bb, L.gs.bb, tol2 >= 1.0 ? 1.0 : 0.0, nrhs, st);
  for (int it = 0; it < maxiter; ++it) {
    const int k = it % m;
    if (k == 0 && it > 0) {
      launch_norm2<T>(r, nh, nrhs, S.sc.red(L.gs.rr, flags), st);
      launch_set_flags(flags, S.outer_flags, S.sc.scal.as<double>(), L.gs.rr, L.gs.bb, tol2, nrhs, st);
      schur(ye, r, bp, 2);  // r = b' - S y_e
    }
    cplx<T>* Wk = Wb + (long)k * dstride;
    schur(r, Wk, r, 1);     // w = S z with z = r
    const bool check_here = !(k == 0 && it > 0);
    launch_gcr_dots<T>(Wb, dstride, Wk, r, k, nh, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.ww, L.gs.alpha,
                       check_here ? L.gs.rr : -1, L.gs.bb, tol2, flags, st);
    launch_gcr_update2<T>(ye, r, r, Wb, Zb, dstride, k, nh, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.alpha, -1,
                          L.gs.bb, tol2, flags, st);
    if ((it + 1) % kCoarseCheck == 0 && it + 1 < maxiter && S.sc.all_flags(L.flag_off, nrhs, st)) break;
  }
  {
    ProfScope ps(S, PK_EO, l, st);
    launch_eo_hop<T>(yo, ye, b, nullptr, Co, L1, L2, nc, 1, 0, 1, 1, nrhs, st);  // b_o - T_oe y_e
  }
  launch_eo_block_apply<T>(x_out, ye, yo, level_MI<T>(L), L1, L2, nc, nrhs, st);
}

// ---- GCR on level l with restarts, stopping per rhs on the recursive
// residual |r| <= tol |b| (device flags; later launches become no-ops).
// precond = false: the coarsest-level solve (z = r);
// precond = true:  a K-cycle level, z = the cycle of level l down to lstop.
template <typename T>
void level_gcr(Solver& S, int l, int lstop, const cplx<T>* b, cplx<T>* x_out, int nrhs, double tol, int maxiter,
               int m, bool precond, hipStream_t st) {
  Level& L = S.lv[l];
  // coarsest level with block-Jacobi preconditioning: GCR on (A M) y = b,
  // then x = M y (not while a batch records its launches)
  const bool jac = !precond && L.jac && current_recorder() == nullptr;
  if (jac && L.eo) {
    eo_gcr<T>(S, l, b, x_out, nrhs, tol, maxiter, m, st);
    return;
  }
  const cplx<T>* Yop = jac ? level_J<T>(L) : nullptr;
  cplx<T>* x = jac ? level_JY<T>(L) : x_out;
  const long n = L.per_rhs();
  const long dstride = n * nrhs;
  Buf* w = L.w<T>();
  cplx<T>* r = w[W_GR].as<cplx<T>>();
  cplx<T>* Zb = L.template Zd<T>().template as<cplx<T>>();
  cplx<T>* Wb = L.template Wd<T>().template as<cplx<T>>();
  int* flags = S.sc.flags.as<int>() + L.flag_off;
  const double tol2 = tol * tol;
  const int check = precond ? 1 : kCoarseCheck;
  const bool recording = current_recorder() != nullptr;
  if (!precond && S.persistent && !recording && L.dof == 16 && !L.fine && (L.nd == 2 || L.nd == 4)) {
    // the whole solve in one cooperative launch
    long nb = (L.V + 15) / 16;
    nb = std::max(8L, std::min((long)S.pcoarse_max_blocks, nb));
    HIPC(hipMemsetAsync(S.pbar.p, 0, sizeof(unsigned) * nrhs, st));
    {
      ProfScope ps(S, PK_COARSE, l, st);
      HIPC(launch_gcr16_persistent<T>(Yop ? Yop : L.Y<T>(), L.cgeom(), b, x, r, Zb, Wb, dstride, m, maxiter, tol2,
                                      nrhs, (int)nb, S.sc.part.as<double>(), S.pbar.as<unsigned>(), S.perr.as<int>(),
                                      S.piters.as<int>(), st, S.pcoarse_coop));
    }
    S.nC += maxiter;  // upper bound of coarse applications (exact count is per rhs on the device)
    if (jac) launch_block_apply<T>(x_out, x, level_MI<T>(L), L.V, L.dof, nrhs, st);
    return;
  }
  launch_fill<T>(x, nullptr, n, nrhs, st);
  launch_fill<T>(r, b, n, nrhs, st);
  launch_norm2<T>(b, n, nrhs, S.sc.red(L.gs.bb), st);
  launch_set_flags(flags, S.outer_flags, S.sc.scal.as<double>(), L.gs.bb, L.gs.bb, tol2 >= 1.0 ? 1.0 : 0.0, nrhs, st);
  // Coarsest level in the three-launch form: the residual norm and stopping
  // flag of each step are taken by the next step's sums kernel, so the
  // update needs no reduction; before a restart the recursive residual is
  // checked explicitly.  The stopping decisions are those of the
  // step-by-step form.
  const bool lag = S.gcr_dots && !precond && !(!L.fine && L.dof == 16 && S.fused_gcr);
  for (int it = 0; it < maxiter; ++it) {
    const int k = it % m;
    if (k == 0 && it > 0) {
      if (lag) {
        launch_norm2<T>(r, n, nrhs, S.sc.red(L.gs.rr, flags), st);
        launch_set_flags(flags, S.outer_flags, S.sc.scal.as<double>(), L.gs.rr, L.gs.bb, tol2, nrhs, st);
      }
      op_apply<T>(S, l, 0, EPI_RESID, x, r, b, nullptr, nrhs, S.sc.red(0, flags), st, Yop);
    }
    cplx<T>* Wk = Wb + (long)k * dstride;
    cplx<T>* Zk = Zb + (long)k * dstride;
    if (!L.fine && L.dof == 16 && S.fused_gcr) {
      // two launches per step: apply + all sums, then the updates
      const cplx<T>* z = r;
      if (precond) {
        vcycle<T>(S, l, lstop, r, Zk, nrhs, st);
        z = Zk;
      }
      {
        ProfScope ps(S, PK_COARSE, l, st);
        CoarseArgs<T> ca;
        ca.out = Wk; ca.in = z; ca.Y = Yop ? Yop : L.Y<T>(); ca.g = L.cgeom(); ca.nrhs = nrhs; ca.red = S.sc.red(0, flags);
        launch_gcr16_apply_dots<T>(ca, r, Wb, dstride, k, L.gs.beta, L.gs.ww, L.gs.alpha, st);
        S.nC += 1;
      }
      launch_gcr_update2<T>(x, r, z, Wb, Zb, dstride, k, n, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.alpha, L.gs.rr,
                            L.gs.bb, tol2, flags, st);
      if (!recording && (it + 1) % check == 0 && it + 1 < maxiter && S.sc.all_flags(L.flag_off, nrhs, st)) break;
      continue;
    }
    if (S.gcr_dots) {
      // three launches per step: apply, all sums, updates
      const cplx<T>* z = r;
      if (precond) {
        vcycle<T>(S, l, lstop, r, Zk, nrhs, st);
        z = Zk;
      }
      op_apply<T>(S, l, 0, EPI_PLAIN, z, Wk, nullptr, nullptr, nrhs, S.sc.red(0, flags), st, Yop);
      const bool check_here = lag && !(k == 0 && it > 0);
      launch_gcr_dots<T>(Wb, dstride, Wk, r, k, n, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.ww, L.gs.alpha,
                         check_here ? L.gs.rr : -1, L.gs.bb, tol2, flags, st);
      launch_gcr_update2<T>(x, r, z, Wb, Zb, dstride, k, n, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.alpha,
                            lag ? -1 : L.gs.rr, L.gs.bb, tol2, flags, st);
      if (!recording && (it + 1) % check == 0 && it + 1 < maxiter && S.sc.all_flags(L.flag_off, nrhs, st)) break;
      continue;
    }
    if (precond) {
      vcycle<T>(S, l, lstop, r, Zk, nrhs, st);
      op_apply<T>(S, l, 0, EPI_PLAIN, Zk, Wk, nullptr, nullptr, nrhs, S.sc.red(0, flags), st);
    } else {
      op_apply<T>(S, l, 0, EPI_PLAIN, r, Wk, nullptr, Zk, nrhs, S.sc.red(0, flags), st, Yop);
    }
    launch_gcr_mdot<T>(Wb, dstride, Wk, k, n, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.ww, st);
    launch_gcr_maxpy<T>(Wk, Zk, Wb, Zb, dstride, r, k, n, nrhs, S.sc.red(0, flags), L.gs.beta, L.gs.ww, L.gs.alpha,
                        st);
    launch_gcr_update<T>(x, r, Zk, Wk, n, nrhs, S.sc.red(0, flags), L.gs.alpha, L.gs.rr, L.gs.bb, tol2, flags, st);
    // Every rhs that met the tolerance turns the remaining launches into
    // no-ops; look at the flags now and then and stop issuing them.  This
    // changes no arithmetic, only how many empty launches are made.
    if (!recording && (it + 1) % check == 0 && it + 1 < maxiter && S.sc.all_flags(L.flag_off, nrhs, st)) break;
  }
  if (jac) launch_block_apply<T>(x_out, x, level_MI<T>(L), L.V, L.dof, nrhs, st);
}

template <typename T>
void coarse_gcr(Solver& S, int l, const cplx<T>* b, cplx<T>* x, int nrhs, hipStream_t st) {
  level_gcr<T>(S, l, l, b, x, nrhs, S.p.coarse_tol, S.p.coarse_maxiter, S.p.coarse_restart, false, st);
}

// ---- V-cycle (five steps listed before Eq. (3), applied to D) ---------------
template <typename T>
void vcycle(Solver& S, int l, int lstop, const cplx<T>* b, cplx<T>* x, int nrhs, hipStream_t st) {
  if (l == lstop) {
    Level& L = S.lv[l];
    if (L.dense && !S.no_dense)
      launch_dense_apply<T>(x, b, Pick<T>::prec == AMG_F64 ? (const cplx<T>*)L.D64.p : (const cplx<T>*)L.D32.p,
                            L.V * L.dof, nrhs, S.outer_flags, st);
    else
      coarse_gcr<T>(S, l, b, x, nrhs, st);
    return;
  }
  Level& L = S.lv[l];
  Level& C = S.lv[l + 1];
  Buf* w = L.w<T>();
  Buf* wc = C.w<T>();
  cplx<T>* r = w[W_R].as<cplx<T>>();
  cplx<T>* p = w[W_P].as<cplx<T>>();
  int pk;
  const void* P = Pstore<T>(S, l, pk);
  const TransferGeom tg = tgeom(S, l, Pick<T>::prec);
  // 1. pre-relax
  mr_smooth<T>(S, l, b, x, r, p, S.p.nu_pre, true, true, nrhs, st);
  // 2. restrict the residual
  cplx<T>* bc = wc[W_B].as<cplx<T>>();
  cplx<T>* xc = wc[W_X].as<cplx<T>>();
  {
    ProfScope ps(S, PK_RESTRICT, l, st);
    launch_restrict<T>(bc, r, P, pk, tg, nrhs, S.outer_flags, st);
  }
  // 3. coarse-level cycle; an intermediate level is a K-cycle when enabled
  if (S.p.kcycle_maxiter > 0 && l + 1 < lstop)
    level_gcr<T>(S, l + 1, lstop, bc, xc, nrhs, S.p.kcycle_tol, S.p.kcycle_maxiter, S.p.kcycle_maxiter, true, st);
  else
    vcycle<T>(S, l + 1, lstop, bc, xc, nrhs, st);
  // 4. coarse-grid correction
  {
    ProfScope ps(S, PK_PROLONG, l, st);
    launch_prolong<T>(x, xc, P, pk, tg, nrhs, 1, S.outer_flags, st);
  }
  // 5. post-relax on the new residual
  op_apply<T>(S, l, 0, EPI_RESID, x, r, b, nullptr, nrhs, S.sc.red(0, S.outer_flags), st);
  mr_smooth<T>(S, l, r, x, r, p, S.p.nu_post, false, false, nrhs, st);
}

// ---- layout helpers ---------------------------------------------------------
// canonical (AoS complex128) <-> internal layout of level l in precision T
template <typename T>
void to_internal(const Solver& S, int l, const double2* canon, cplx<T>* out, int nrhs, hipStream_t st) {
  const Level& L = S.lv[l];
  launch_convert<double, T>(out, canon, L.V, L.dof, L.dof, L.lay<T>().W, nrhs, st);
}
template <typename T>
void to_canonical(const Solver& S, int l, const cplx<T>* in, double2* canon, int nrhs, hipStream_t st) {
  const Level& L = S.lv[l];
  launch_convert<T, double>(canon, in, L.V, L.dof, L.lay<T>().W, L.dof, nrhs, st);
}

// ---- setup ------------------------------------------------------------------
// Dense inverse of the operator of coarse level l (the exact coarsest
// solve) when the finished level, with all its near-null vectors, has at
// most coarse_dense_max unknowns; the adaptive setup's partial levels follow
// the finished level's choice.  Otherwise the level is solved by GCR when it
// is the coarsest one of a cycle.
void build_dense(Solver& S, int l, hipStream_t st) {
  Level& L = S.lv[l];
  const long N = L.V * L.dof;
  L.dense = false;
  if (L.fine || L.V * (long)L.dof_max > S.p.coarse_dense_max) return;
  const size_t nn = (size_t)N * N;
  S.gjA.ensure(nn * sizeof(double2));
  S.gjB.ensure(nn * sizeof(double2));
  S.gjkey.ensure((size_t)(N + 2) * sizeof(unsigned long long));
  S.gjint.ensure((size_t)(3 * N + 8) * sizeof(int));
  L.D64.ensure(nn * sizeof(double2));
  const bool f32 = S.p.inner_prec == AMG_F32;
  if (f32) L.D32.ensure(nn * sizeof(float2));
  int* piv = S.gjint.as<int>();
  int* used = piv + N;
  int* pinv = used + N;
  int* err = pinv + N;
  launch_dense_assemble(S.gjA.as<double2>(), L.Y64.as<double2>(), L.cgeom(), st);
  launch_gj_invert(S.gjA.as<double2>(), S.gjB.as<double2>(), N, S.gjkey.as<unsigned long long>(), piv, used, pinv,
                   err, L.D64.as<double2>(), f32 ? L.D32.as<float2>() : nullptr, st);
  int herr = 0;
  HIPC(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (herr) fail(AMG_ERR_SINGULAR, "the operator of level " + std::to_string(l) + " is singular (exact coarsest solve)");
  L.dense = true;
}

// Block-Jacobi data of a coarse level that GCR solves as the coarsest level:
// M = the inverse of every site's diagonal block and the stencil of A M.
// A singular diagonal block leaves the level with plain GCR.
void build_jacobi(Solver& S, int l, hipStream_t st) {
  Level& L = S.lv[l];
  L.jac = false;
  L.eo = false;
  L.s9 = false;
  if (!S.p.coarse_jacobi || L.fine || L.dense || !block_jacobi_supported(L.dof)) return;
  const int ndir = L.ndir();
  const long per = (long)L.dof_max * L.dof_max;
  const long n_m = L.V * (long)L.dof * L.dof;
  const bool f32 = S.p.inner_prec == AMG_F32;
  L.MI64.ensure(L.V * per * sizeof(double2));
  L.J64.ensure(L.V * ndir * per * sizeof(double2));
  if (f32) {
    L.MI32.ensure(L.V * per * sizeof(float2));
    L.J32.ensure(L.V * ndir * per * sizeof(float2));
  }
  S.jerr.ensure(sizeof(int));
  int* err = S.jerr.as<int>();
  HIPC(hipMemsetAsync(err, 0, sizeof(int), st));
  launch_block_inverse(L.MI64.as<double2>(), L.Y64.as<double2>(), L.V, ndir, L.dof, err, st);
  HIPC(hipGetLastError());  // (the 48-wide kernel takes 72 KB of LDS per block)
  launch_jacobi_couplings(L.J64.as<double2>(), L.Y64.as<double2>(), L.MI64.as<double2>(), L.cgeom(), st);
  if (f32) {
    launch_p_convert(L.MI32.p, P_F32, L.MI64.as<double2>(), n_m, st);
    launch_p_convert(L.J32.p, P_F32, L.J64.as<double2>(), n_m * ndir, st);
  }
  L.eo = false;
  if (S.p.coarse_eo && eo_supported(L.nd, L.dims, L.dof)) {
    const long csz = L.V * 2 * (long)L.dof_max * L.dof_max;  // half the sites x 4 directions
    L.CE64.ensure(csz * sizeof(double2));
    L.CO64.ensure(csz * sizeof(double2));
    launch_eo_split(L.CE64.as<double2>(), L.CO64.as<double2>(), L.J64.as<double2>(), L.dims[0], L.dims[1], L.dof, st);
    if (f32) {
      L.CE32.ensure(csz * sizeof(float2));
      L.CO32.ensure(csz * sizeof(float2));
      const long nsplit = L.V * 2 * (long)L.dof * L.dof;
      launch_p_convert(L.CE32.p, P_F32, L.CE64.as<double2>(), nsplit, st);
      launch_p_convert(L.CO32.p, P_F32, L.CO64.as<double2>(), nsplit, st);
    }
    if (L.dof == 16) {
      const long ssz = L.V / 2 * 9 * 256;
      L.SE64.ensure(ssz * sizeof(double2));
      launch_eo_schur_build(L.SE64.as<double2>(), L.CE64.as<double2>(), L.CO64.as<double2>(), L.dims[0], L.dims[1],
                            16, st);
      if (f32) {
        L.SE32.ensure(ssz * sizeof(float2));
        launch_p_convert(L.SE32.p, P_F32, L.SE64.as<double2>(), ssz, st);
      }
    }
  }
  int herr = 0;
  HIPC(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  L.jac = herr == 0;
  L.eo = L.jac && S.p.coarse_eo && eo_supported(L.nd, L.dims, L.dof);
  L.s9 = L.eo && L.dof == 16;
}

// Build P_l from the first L.nv raw vectors and A_{l+1} = P_l^dag A_l P_l.
void build_transfer(Solver& S, int l, hipStream_t st) {
  Level& F = S.lv[l];
  Level& C = S.lv[l + 1];
  const int nv = F.nv;
  C.dof = 2 * nv;
  C.lay64 = Layout{C.V, C.dof, C.dof};
  C.lay32 = C.lay64;
  const TransferGeom tg = tgeom(S, l, AMG_F64);
  const long psz = (long)F.V * F.dof * nv;  // P entries
  // buffers are sized for the final number of vectors on first use: the
  // adaptive setup rebuilds the transfer once per added vector, and growing
  // a buffer (hipFree + hipMalloc) synchronises the device every time
  const int nvm = std::max(nv, F.nv_max);
  const long psz_max = (long)F.V * F.dof * nvm;
  F.P64.ensure(psz_max * sizeof(double2));
  int* err = S.sc.flags.as<int>() + S.flags_base;  // scratch flag
  HIPC(hipMemsetAsync(err, 0, sizeof(int), st));
  launch_orthonormalise(F.P64.as<double2>(), F.vecs.as<double2>(), tg, err, st);
  int herr = 0;
  HIPC(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (herr) fail(AMG_ERR_RANK, "near-null vectors are linearly dependent on a block (level " + std::to_string(l) + ")");
  if (S.p.inner_prec == AMG_F32) {
    if (S.p.p_bf16) {
      launch_p_roundtrip_bf16(F.P64.as<double2>(), psz, st);
      F.Pbf.ensure(psz_max * sizeof(bf16x2));
      launch_p_convert(F.Pbf.p, P_BF16, F.P64.as<double2>(), psz, st);
    } else {
      F.P32.ensure(psz_max * sizeof(float2));
      launch_p_convert(F.P32.p, P_F32, F.P64.as<double2>(), psz, st);
    }
  }
  // Galerkin product column by column: E = unit coarse fields, F = P E,
  // S = split(A F), R = P^dag S, scattered into Y.  Mass matrix likewise.
  const int nc = C.dof, ndir = F.ndir();
  const int ncm = 2 * nvm;
  const long ysz = C.V * ndir * (long)nc * nc;
  C.Y64.ensure(C.V * ndir * (long)ncm * ncm * sizeof(double2));
  C.M64.ensure(C.V * (long)ncm * ncm * sizeof(double2));
  const long fper = F.per_rhs();
  const long budget = 1L << 31;  // bytes for the split outputs
  auto chunk_of = [&](int c) {
    int ch = c;
    while (ch > 1 && (long)ch * ndir * fper * 16 > budget) ch = (ch + 1) / 2;
    return ch;
  };
  const int chunk = chunk_of(nc);
  const size_t chm = (size_t)std::max(chunk, chunk_of(ncm));
  S.tE.ensure(chm * C.V * ncm * sizeof(double2));
  S.tF.ensure(chm * fper * sizeof(double2));
  S.tS.ensure(chm * ndir * fper * sizeof(double2));
  S.tR.ensure(chm * ndir * C.V * ncm * sizeof(double2));
  double2* E = S.tE.as<double2>();
  double2* Fv = S.tF.as<double2>();
  double2* Sv = S.tS.as<double2>();
  double2* Rv = S.tR.as<double2>();
  for (int t0 = 0; t0 < nc; t0 += chunk) {
    const int ch = std::min(chunk, nc - t0);
    launch_unit_coarse(E, C.V, nc, t0, ch, st);
    launch_prolong<double>(Fv, E, F.P64.p, P_F64, tg, ch, 0, nullptr, st);
    if (F.fine) {
      const amg_gauge& g = *S.g;
      if (g.nd == 2)
        launch_wilson2d_split(Sv, Fv, g.U64.as<double2>(), S.mass, g.dims[0], g.dims[1], F.blk[0], F.blk[1], ch, st);
      else
        launch_wilson4d_split(Sv, Fv, g.U64.as<double2>(), S.mass, g.dims, F.blk, ch, st);
    } else {
      launch_coarse_split(Sv, Fv, F.Y64.as<double2>(), F.cgeom(), F.blk, ch, st);
    }
    launch_restrict<double>(Rv, Sv, F.P64.p, P_F64, tg, ndir * ch, nullptr, st);
    launch_galerkin_scatter(C.Y64.as<double2>(), Rv, C.V, nc, ndir, t0, ch, st);
    // mass matrix: fine level d(D)/dm = 1, coarse levels their own M
    const double2* MF = Fv;
    if (!F.fine) {
      launch_coarse_massmat(Sv, Fv, F.M64.as<double2>(), F.cgeom(), ch, st);
      MF = Sv;
    }
    launch_restrict<double>(Rv, MF, F.P64.p, P_F64, tg, ch, nullptr, st);
    launch_galerkin_scatter(C.M64.as<double2>(), Rv, C.V, nc, 1, t0, ch, st);
  }
  if (S.p.inner_prec == AMG_F32) {
    C.Y32.ensure(C.V * ndir * (long)ncm * ncm * sizeof(float2));
    launch_p_convert(C.Y32.p, P_F32, C.Y64.as<double2>(), ysz, st);
  }
  build_dense(S, l + 1, st);
  // block-Jacobi data only for a level that can be the coarsest of a cycle:
  // the last level, or the next level while the adaptive setup is still
  // adding vectors (its sweeps stop the cycle there)
  if (l + 2 == (int)S.lv.size() || F.nv < F.nv_max) {
    build_jacobi(S, l + 1, st);
  } else {
    C.jac = C.eo = C.s9 = false;
  }
}

void check_params(const amg_gauge* g, const amg_mg_params* p) {
  if (!g || !p) fail(AMG_ERR_ARG, "NULL gauge or params");
  if (p->nlevels < 2 || p->nlevels > 4) fail(AMG_ERR_ARG, "nlevels must be 2..4");
  if (p->nu_pre < 0 || p->nu_post < 0 || p->nu_pre > 64 || p->nu_post > 64) fail(AMG_ERR_ARG, "bad smoothing steps");
  if (!(p->omega > 0.0 && p->omega < 2.0)) fail(AMG_ERR_ARG, "omega must be in (0, 2)");
  if (!(p->coarse_tol >= 0.0) || !std::isfinite(p->coarse_tol)) fail(AMG_ERR_ARG, "bad coarse_tol");
  if (p->coarse_maxiter < 1 || p->coarse_restart < 1 || p->coarse_restart > GCR_KMAX) fail(AMG_ERR_ARG, "bad coarse GCR limits");
  if (p->outer_restart < 1 || p->outer_restart > GCR_KMAX) fail(AMG_ERR_ARG, "outer_restart must be 1..32");
  if (p->inner_prec != AMG_F64 && p->inner_prec != AMG_F32) fail(AMG_ERR_ARG, "bad inner_prec");
  if (p->kcycle_maxiter < 0 || p->kcycle_maxiter > GCR_KMAX) fail(AMG_ERR_ARG, "kcycle_maxiter must be 0..32");
  if (p->kcycle_maxiter > 0 && !(p->kcycle_tol >= 0.0 && std::isfinite(p->kcycle_tol))) fail(AMG_ERR_ARG, "bad kcycle_tol");
  if (p->coarse_jacobi != 0 && p->coarse_jacobi != 1) fail(AMG_ERR_ARG, "coarse_jacobi must be 0 or 1");
  if (p->coarse_eo != 0 && p->coarse_eo != 1) fail(AMG_ERR_ARG, "coarse_eo must be 0 or 1");
  if (p->coarse_eo && !p->coarse_jacobi) fail(AMG_ERR_ARG, "coarse_eo needs coarse_jacobi");
  if (p->coarse_dense_max < 0 || p->coarse_dense_max > AMG_DENSE_MAX)
    fail(AMG_ERR_ARG, "coarse_dense_max must be 0.." + std::to_string(AMG_DENSE_MAX));
  int dims[4];
  for (int mu = 0; mu < 4; ++mu) dims[mu] = g->dims[mu];
  int dof = g->dof;
  for (int l = 0; l + 1 < p->nlevels; ++l) {
    if (p->nvec[l] < 1 || p->nvec[l] > 64) fail(AMG_ERR_ARG, "nvec must be 1..64");
    for (int mu = 0; mu < g->nd; ++mu) {
      const int b = p->block[l][mu];
      if (b < 1 || dims[mu] % b) fail(AMG_ERR_SHAPE, "block extents must divide the lattice extents");
      dims[mu] /= b;
    }
    dof = 2 * p->nvec[l];
  }
  (void)dof;
}

Solver* new_solver(const amg_gauge* g, const amg_mg_params* p) {
  check_params(g, p);
  Solver* S = new Solver();
  S->g = g;
  S->p = *p;
  S->mass = g->mass;
  S->lv.resize(p->nlevels);
  for (int l = 0; l < p->nlevels; ++l) {
    Level& L = S->lv[l];
    L.nd = g->nd;
    if (l == 0) {
      L.fine = true;
      for (int mu = 0; mu < 4; ++mu) L.dims[mu] = g->dims[mu];
      L.V = g->V;
      L.dof = L.dof_max = g->dof;
      L.lay64 = Layout{L.V, L.dof, 1};
      L.lay32 = Layout{L.V, L.dof, 2};
    } else {
      Level& F = S->lv[l - 1];
      L.V = 1;
      for (int mu = 0; mu < 4; ++mu) {
        L.dims[mu] = mu < g->nd ? F.dims[mu] / p->block[l - 1][mu] : 1;
        L.V *= L.dims[mu];
      }
      L.dof = L.dof_max = 2 * p->nvec[l - 1];
      L.lay64 = L.lay32 = Layout{L.V, L.dof, L.dof};
    }
    if (l + 1 < p->nlevels) {
      L.has_next = true;
      for (int mu = 0; mu < 4; ++mu) L.blk[mu] = mu < g->nd ? p->block[l][mu] : 1;
      L.nv = L.nv_max = p->nvec[l];
    }
  }
  // scalar slots: per level MR alpha + GCR set; outer GCR set
  int off = 0;
  for (auto& L : S->lv) {
    L.mr_slot = off;
    off += 2 * RHS_MAX;
    L.gs.at(off);
    off += GcrSlots::size();
  }
  S->og.at(off);
  off += GcrSlots::size();
  const int nflags = RHS_MAX * ((int)S->lv.size() + 2);
  for (size_t l = 0; l < S->lv.size(); ++l) S->lv[l].flag_off = RHS_MAX * (int)l;
  S->flags_base = RHS_MAX * (int)S->lv.size();
  S->sc.init(off, nflags);
  S->pbar.ensure(sizeof(unsigned) * RHS_MAX);
  S->perr.ensure(sizeof(int) * 4);
  S->piters.ensure(sizeof(int) * RHS_MAX);
  HIPC(hipMemset(S->perr.p, 0, sizeof(int) * 4));
  if (const char* e = std::getenv("AMG_PERSISTENT_COARSE")) S->persistent = std::atoi(e) != 0;
  if (const char* e = std::getenv("AMG_PCOARSE_BLOCKS")) S->pcoarse_max_blocks = std::max(1, std::min(256, std::atoi(e)));
  if (const char* e = std::getenv("AMG_PCOARSE_COOP")) S->pcoarse_coop = std::atoi(e) != 0;
  if (const char* e = std::getenv("AMG_FUSED_GCR")) S->fused_gcr = std::atoi(e) != 0;
  if (const char* e = std::getenv("AMG_GCR_DOTS")) S->gcr_dots = std::atoi(e) != 0;
  if (const char* e = std::getenv("AMG_MRHS_MIN")) S->mrhs_min = std::max(1, std::atoi(e));
  return S;
}

void upload_vectors(Solver& S, int l, const void* dev_canon, int nv, hipStream_t st) {
  Level& L = S.lv[l];
  L.vecs.ensure((size_t)L.nv_max * L.V * L.dof * sizeof(double2));
  to_internal<double>(S, l, (const double2*)dev_canon, L.vecs.as<double2>(), nv, st);
}

// nu0 MR steps on A v = 0 from v (in place), FP64, on level l
void relax_homogeneous(Solver& S, int l, double2* v, int nu0, hipStream_t st) {
  Level& L = S.lv[l];
  const long n = L.per_rhs();
  double2* r = L.w64[W_R].as<double2>();
  double2* p = L.w64[W_P].as<double2>();
  double2* z = S.tzero.as<double2>();
  op_apply<double>(S, l, 0, EPI_RESID, v, r, z, nullptr, 1, S.sc.red(0), st);  // r = 0 - A v
  for (int i = 0; i < nu0; ++i) {
    op_apply<double>(S, l, 0, EPI_MRDOT, r, p, nullptr, nullptr, 1, S.sc.red(L.mr_slot, nullptr, S.p.omega), st);
    launch_mr_update<double>(v, r, r, p, S.sc.scal.as<double>() + L.mr_slot, n, 1, 0, 1, nullptr, st);
  }
}

// Vectors k0.. of level l each get ncyc sweeps of the two-level error
// propagation e <- e - V(A_l e), V built from the vectors before them, and
// are normalised; finally P_l and A_{l+1} are built from all of them (the
// adaptive procedure after Eq. (5)).  Vectors before k0 are used as given.
void adaptive_sweeps(Solver& S, int l, int ncyc, int k0, hipStream_t st) {
  Level& L = S.lv[l];
  const int nv = L.nv_max;
  const long n = L.per_rhs();
  double2* vecs = L.vecs.as<double2>();
  double2* t = L.w64[W_B].as<double2>();  // A e
  double2* zc = S.otmp.as<double2>();
  for (int k = k0; k < nv; ++k) {
    L.nv = k;
    build_transfer(S, l, st);
    double2* e = vecs + (long)k * n;
    for (int c = 0; c < ncyc; ++c) {
      op_apply<double>(S, l, 0, EPI_PLAIN, e, t, nullptr, nullptr, 1, S.sc.red(0), st);
      // z = V(A e) with level l+1 as the coarsest; kept in the outer scratch
      // (level l's own x buffer is written inside the cycle)
      vcycle<double>(S, l, l + 1, t, zc, 1, st);
      launch_axpy<double>(e, zc, -1.0, 0.0, n, 1, st);
    }
    launch_norm2<double>(e, n, 1, S.sc.red(L.gs.rr), st);
    launch_scale_inv_norm<double>(e, S.sc.scal.as<double>() + L.gs.rr, n, 1, st);
  }
  L.nv = nv;
  build_transfer(S, l, st);
}

void zero_scratch(Solver& S, int l, hipStream_t st) {
  const long n = S.lv[l].per_rhs();
  S.tzero.ensure(n * sizeof(double2));
  HIPC(hipMemsetAsync(S.tzero.p, 0, n * sizeof(double2), st));
}

// Adaptive setup of coarsening l from random vectors: the first relaxed by
// nu0 MR steps on A_l v = 0 (Eq. (4)), the others by the sweeps above.
void adaptive_level(Solver& S, int l, const void* dev_init, int nu0, int ncyc, hipStream_t st) {
  Level& L = S.lv[l];
  upload_vectors(S, l, dev_init, L.nv_max, st);
  zero_scratch(S, l, st);
  relax_homogeneous(S, l, L.vecs.as<double2>(), nu0, st);
  adaptive_sweeps(S, l, ncyc, 1, st);
}

// Coarsening l from n_start given vectors (proposals), each relaxed by nu MR
// steps on A_l v = 0; the remaining nvec - n_start vectors are built by the
// adaptive procedure (ncyc sweeps each) from the first random vectors of
// dev_rand.
void refined_level(Solver& S, int l, const void* dev_start, int n_start, int nu, const void* dev_rand, int ncyc,
                   hipStream_t st) {
  Level& L = S.lv[l];
  const long n = L.per_rhs();
  upload_vectors(S, l, dev_start, n_start, st);
  if (n_start < L.nv_max)
    to_internal<double>(S, l, (const double2*)dev_rand, L.vecs.as<double2>() + (long)n_start * n, L.nv_max - n_start,
                        st);
  zero_scratch(S, l, st);
  if (nu > 0)
    for (int k = 0; k < n_start; ++k) relax_homogeneous(S, l, L.vecs.as<double2>() + (long)k * n, nu, st);
  adaptive_sweeps(S, l, ncyc, n_start, st);
}

// ---- convergence factor of the method as a stationary iteration ----------------
// e <- e - M(D e) from e0 (canonical); returns (|e_n| / |e_0|)^(1/n).
void precondition(Solver& S, const double2* r, double2* z, int nrhs, hipStream_t st);

double mg_convergence(Solver& S, const double2* e0, int iters, hipStream_t st) {
  ensure_work(S, 1);
  Level& F = S.lv[0];
  const long n = F.per_rhs();
  double2* e = S.ox.as<double2>();
  double2* t = S.ob.as<double2>();
  double2* z = S.otmp.as<double2>();
  const int slot = S.og.rr;
  to_internal<double>(S, 0, e0, e, 1, st);
  launch_norm2<double>(e, n, 1, S.sc.red(slot), st);
  const double n0 = S.sc.fetch(slot, 1, st)[0];
  if (!(n0 > 0.0) || !std::isfinite(n0)) fail(AMG_ERR_ARG, "starting error must be finite and nonzero");
  for (int i = 0; i < iters; ++i) {
    op_apply<double>(S, 0, 0, EPI_PLAIN, e, t, nullptr, nullptr, 1, S.sc.red(0), st);
    precondition(S, t, z, 1, st);
    launch_axpy<double>(e, z, -1.0, 0.0, n, 1, st);
  }
  launch_norm2<double>(e, n, 1, S.sc.red(slot), st);
  const double n1 = S.sc.fetch(slot, 1, st)[0];
  if (!std::isfinite(n1)) fail(AMG_ERR_NAN, "non-finite error in the convergence test");
  return std::pow(std::sqrt(n1 / n0), 1.0 / iters);
}

// ---- outer FGCR (fine level, FP64) ------------------------------------------
struct OuterResult {
  int iters = 0;
  bool conv = false;
  std::vector<double> rel;
};

void precondition(Solver& S, const double2* r, double2* z, int nrhs, hipStream_t st) {
  const int last = (int)S.lv.size() - 1;
  if (S.p.inner_prec == AMG_F64) {
    vcycle<double>(S, 0, last, r, z, nrhs, st);
  } else {
    Level& F = S.lv[0];
    float2* r32 = F.w32[W_B].as<float2>();
    float2* z32 = F.w32[W_X].as<float2>();
    launch_convert<double, float>(r32, r, F.V, F.dof, F.lay64.W, F.lay32.W, nrhs, st);
    vcycle<float>(S, 0, last, r32, z32, nrhs, st);
    launch_convert<float, double>(z, z32, F.V, F.dof, F.lay32.W, F.lay64.W, nrhs, st);
  }
}

OuterResult fgcr_outer(Solver& S, const double2* b, double2* x, int nrhs, double tol, int maxiter, hipStream_t st) {
  Level& F = S.lv[0];
  const long n = F.per_rhs();
  const long dstride = n * nrhs;
  double2* r = S.orr.as<double2>();
  double2* Zb = S.oZ.as<double2>();
  double2* Wb = S.oW.as<double2>();
  const int m = S.p.outer_restart;
  const GcrSlots& gs = S.og;
  launch_fill<double>(x, nullptr, n, nrhs, st);
  launch_fill<double>(r, b, n, nrhs, st);
  launch_norm2<double>(b, n, nrhs, S.sc.red(gs.bb), st);
  launch_norm2<double>(r, n, nrhs, S.sc.red(gs.rr), st);
  std::vector<double> bb(nrhs), rr(nrhs);
  {
    const double* h = S.sc.fetch(gs.bb, nrhs, st);
    for (int i = 0; i < nrhs; ++i) bb[i] = h[i];
  }
  for (int i = 0; i < nrhs; ++i)
    if (!std::isfinite(bb[i])) fail(AMG_ERR_NAN, "right-hand side " + std::to_string(i) + " has non-finite entries");
  OuterResult res;
  int k = 0;
  auto read_rr = [&]() {
    const double* h = S.sc.fetch(gs.rr, nrhs, st);
    for (int i = 0; i < nrhs; ++i) rr[i] = h[i];
  };
  auto all_below = [&]() {
    for (int i = 0; i < nrhs; ++i)
      if (!(rr[i] <= tol * tol * bb[i])) return false;
    return true;
  };
  auto true_residual = [&]() {
    op_apply<double>(S, 0, 0, EPI_RESID, x, r, b, nullptr, nrhs, S.sc.red(0), st);
    launch_norm2<double>(r, n, nrhs, S.sc.red(gs.rr), st);
  };
  read_rr();
  for (;;) {
    if (all_below()) {
      true_residual();
      read_rr();
      if (all_below()) { res.conv = true; break; }
      k = 0;
    }
    if (res.iters >= maxiter) break;
    double2* Zk = Zb + (long)k * dstride;
    double2* Wk = Wb + (long)k * dstride;
    precondition(S, r, Zk, nrhs, st);
    op_apply<double>(S, 0, 0, EPI_PLAIN, Zk, Wk, nullptr, nullptr, nrhs, S.sc.red(0), st);
    launch_gcr_mdot<double>(Wb, dstride, Wk, k, n, nrhs, S.sc.red(0), gs.beta, gs.ww, st);
    launch_gcr_maxpy<double>(Wk, Zk, Wb, Zb, dstride, r, k, n, nrhs, S.sc.red(0), gs.beta, gs.ww, gs.alpha, st);
    launch_gcr_update<double>(x, r, Zk, Wk, n, nrhs, S.sc.red(0), gs.alpha, gs.rr, gs.bb, 0.0, nullptr, st);
    res.iters++;
    k++;
    if (k == m) {
      true_residual();
      k = 0;
    }
    read_rr();
  }
  if (!res.conv) {
    true_residual();
    read_rr();
  }
  res.rel.resize(nrhs);
  for (int i = 0; i < nrhs; ++i) res.rel[i] = bb[i] > 0 ? std::sqrt(rr[i] / bb[i]) : 0.0;
  return res;
}

// A persistent coarse solve whose grid barrier timed out has left the flag set.
void check_persistent(Solver& S) {
  int e = 0;
  HIPC(hipMemcpy(&e, S.perr.p, sizeof(int), hipMemcpyDeviceToHost));
  if (e) {
    HIPC(hipMemset(S.perr.p, 0, sizeof(int)));
    fail(AMG_ERR_HIP, "a grid barrier of the persistent coarsest solve timed out");
  }
}

void check_ptr(const void* p, const char* what) {
  if (!p) fail(AMG_ERR_ARG, std::string("NULL ") + what);
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

// ===========================================================================
// Batched solves: many independent solvers, one launch per stage.
//
// The solve of each instance is recorded (the same host code as a single
// solve, with host-side checks off and every copy / clear done by kernels),
// the recordings are merged stage by stage into batched launches (argument
// structs in a device array, instance = blockIdx.z), and each segment of the
// outer iteration is captured once into a HIP graph.  Right-hand sides that
// have converged are masked on the device by their instance's outer flags.
// ===========================================================================
struct amg_batch {
  std::vector<Solver*> S;
  std::vector<int> nrhs;
  int n = 0, m = 0, red_cap = RED_MAX_BLOCKS;
  int mrhs = 1;  // coarse levels on the multi-rhs MFMA kernel (1) or the per-rhs stencil (0)
  struct Trial {
    int red_cap, mrhs;
    float ms;  // one batched outer iteration
  };
  std::vector<Trial> trials;  // the autotuner's candidates
  hipStream_t st = nullptr;
  Buf args_dev, flags_dev, gath_dev;
  double* gath_host = nullptr;
  int* flags_host = nullptr;
  struct Op {
    const void* fn;
    dim3 grid, block;
    size_t off;
    std::vector<char> a0;
  };
  struct Seg {
    std::vector<Op> ops;
    hipGraphExec_t exec = nullptr;
  };
  Seg init, truer;
  std::vector<Seg> iters;
  std::vector<char> img;
  ~amg_batch() {
    auto drop = [](Seg& g) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    };
    drop(init);
    drop(truer);
    for (auto& g : iters) drop(g);
    if (gath_host) (void)hipHostFree(gath_host);
    if (flags_host) (void)hipHostFree(flags_host);
    if (st) (void)hipStreamDestroy(st);
    for (Solver* s : S) {
      s->outer_flags = nullptr;
      s->no_dense = false;
    }
  }
};

namespace {

using Batch = amg_batch;

// record fn(S_i, i) for every instance and merge the launches stage by stage
template <class F>
void batch_record(Batch& B, Batch::Seg& seg, F fn) {
  std::vector<Recorder> recs(B.n);
  for (int i = 0; i < B.n; ++i) {
    current_recorder() = &recs[i];
    try {
      fn(*B.S[i], i);
    } catch (...) {
      current_recorder() = nullptr;
      throw;
    }
    current_recorder() = nullptr;
  }
  const size_t nops = recs[0].ops.size();
  for (int i = 1; i < B.n; ++i)
    if (recs[i].ops.size() != nops) fail(AMG_ERR_STATE, "batched instances record different launch sequences");
  seg.ops.clear();
  for (size_t j = 0; j < nops; ++j) {
    Batch::Op op;
    const RecordedLaunch& r0 = recs[0].ops[j];
    op.fn = r0.fn;
    op.block = r0.block;
    op.grid = dim3(1, 1, (unsigned)B.n);
    const size_t asz = r0.args.size();
    size_t off = (B.img.size() + 255) & ~size_t(255);
    B.img.resize(off + asz * B.n);
    for (int i = 0; i < B.n; ++i) {
      const RecordedLaunch& r = recs[i].ops[j];
      if (r.fn != op.fn || r.args.size() != asz || r.block.x != op.block.x)
        fail(AMG_ERR_STATE, "batched instances record different kernels at one stage");
      op.grid.x = std::max(op.grid.x, r.grid.x);
      op.grid.y = std::max(op.grid.y, r.grid.y);
      std::memcpy(B.img.data() + off + asz * i, r.args.data(), asz);
    }
    op.off = off;
    op.a0 = r0.args;
    seg.ops.push_back(std::move(op));
  }
}

void batch_capture(Batch& B, Batch::Seg& seg) {
  hipGraph_t g = nullptr;
  HIPC(hipStreamBeginCapture(B.st, hipStreamCaptureModeThreadLocal));
  for (auto& op : seg.ops) {
    void* dptr = static_cast<char*>(B.args_dev.p) + op.off;
    void* kargs[2] = {op.a0.data(), &dptr};
    const hipError_t e = hipLaunchKernel(op.fn, op.grid, op.block, kargs, 0, B.st);
    if (e != hipSuccess) {
      hipGraph_t dummy = nullptr;
      (void)hipStreamEndCapture(B.st, &dummy);
      if (dummy) (void)hipGraphDestroy(dummy);
      hip_check(e, "hipLaunchKernel (capture)");
    }
  }
  HIPC(hipStreamEndCapture(B.st, &g));
  const hipError_t e = hipGraphInstantiate(&seg.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hip_check(e, "hipGraphInstantiate");
}

// segments of the batched outer FGCR (fine level, FP64); gathered scalars:
// rr of instance i at gath[i * RHS_MAX], bb at gath[(n + i) * RHS_MAX]
void batch_build(Batch& B) {
  B.img.clear();
  B.iters.assign(B.m, Batch::Seg());
  double* gath = B.gath_dev.as<double>();
  auto rr_out = [&](int i) { return gath + (long)i * RHS_MAX; };
  auto bb_out = [&](int i) { return gath + (long)(B.n + i) * RHS_MAX; };
  batch_record(B, B.init, [&](Solver& S, int i) {
    const long n = S.lv[0].per_rhs();
    const int nr = B.nrhs[i];
    double2* b = S.ob.as<double2>();
    launch_fill<double>(S.ox.as<double2>(), nullptr, n, nr, B.st);
    launch_fill<double>(S.orr.as<double2>(), b, n, nr, B.st);
    launch_norm2<double>(b, n, nr, S.sc.red(S.og.bb), B.st);
    launch_norm2<double>(S.orr.as<double2>(), n, nr, S.sc.red(S.og.rr), B.st);
    launch_gather(bb_out(i), S.sc.scal.as<double>(), S.og.bb, nr, B.st);
    launch_gather(rr_out(i), S.sc.scal.as<double>(), S.og.rr, nr, B.st);
  });
  for (int k = 0; k < B.m; ++k)
    batch_record(B, B.iters[k], [&](Solver& S, int i) {
      const long n = S.lv[0].per_rhs();
      const int nr = B.nrhs[i];
      const long dstride = n * nr;
      double2* r = S.orr.as<double2>();
      double2* x = S.ox.as<double2>();
      double2* Zb = S.oZ.as<double2>();
      double2* Wb = S.oW.as<double2>();
      double2* Zk = Zb + (long)k * dstride;
      double2* Wk = Wb + (long)k * dstride;
      const GcrSlots& gs = S.og;
      precondition(S, r, Zk, nr, B.st);
      op_apply<double>(S, 0, 0, EPI_PLAIN, Zk, Wk, nullptr, nullptr, nr, S.sc.red(0, S.outer_flags), B.st);
      launch_gcr_mdot<double>(Wb, dstride, Wk, k, n, nr, S.sc.red(0, S.outer_flags), gs.beta, gs.ww, B.st);
      launch_gcr_maxpy<double>(Wk, Zk, Wb, Zb, dstride, r, k, n, nr, S.sc.red(0, S.outer_flags), gs.beta, gs.ww,
                               gs.alpha, B.st);
      launch_gcr_update<double>(x, r, Zk, Wk, n, nr, S.sc.red(0, S.outer_flags), gs.alpha, gs.rr, gs.bb, 0.0, nullptr,
                                B.st);
      launch_gather(rr_out(i), S.sc.scal.as<double>(), gs.rr, nr, B.st);
    });
  batch_record(B, B.truer, [&](Solver& S, int i) {
    const long n = S.lv[0].per_rhs();
    const int nr = B.nrhs[i];
    op_apply<double>(S, 0, 0, EPI_RESID, S.ox.as<double2>(), S.orr.as<double2>(), S.ob.as<double2>(), nullptr, nr,
                     S.sc.red(0), B.st);
    launch_norm2<double>(S.orr.as<double2>(), n, nr, S.sc.red(S.og.rr), B.st);
    launch_gather(rr_out(i), S.sc.scal.as<double>(), S.og.rr, nr, B.st);
  });
  B.args_dev.ensure(std::max<size_t>(B.img.size(), 256));
  HIPC(hipMemcpy(B.args_dev.p, B.img.data(), B.img.size(), hipMemcpyHostToDevice));
  batch_capture(B, B.init);
  for (auto& g : B.iters) batch_capture(B, g);
  batch_capture(B, B.truer);
}

void batch_replay(Batch& B, Batch::Seg& seg) { HIPC(hipGraphLaunch(seg.exec, B.st)); }

void batch_fetch(Batch& B) {
  HIPC(hipMemcpyAsync(B.gath_host, B.gath_dev.p, sizeof(double) * 2 * B.n * RHS_MAX, hipMemcpyDeviceToHost, B.st));
  HIPC(hipStreamSynchronize(B.st));
}

void batch_put_flags(Batch& B) {
  HIPC(hipMemcpyAsync(B.flags_dev.p, B.flags_host, sizeof(int) * B.n * RHS_MAX, hipMemcpyHostToDevice, B.st));
}

struct BatchResult {
  std::vector<int> iters;
  std::vector<double> rel;
  std::vector<int> done;
  int outer = 0;
};

BatchResult batch_run(Batch& B, double tol, int maxiter) {
  const int n = B.n;
  std::vector<int> base(n + 1, 0);
  for (int i = 0; i < n; ++i) base[i + 1] = base[i] + B.nrhs[i];
  const int tot = base[n];
  BatchResult R;
  R.iters.assign(tot, 0);
  R.rel.assign(tot, 0.0);
  std::vector<int> state(tot, 0);  // 0 active, 1 candidate (recursive residual below tol), 2 done
  std::vector<double> bb(tot);
  auto rr = [&](int i, int j) { return B.gath_host[(long)i * RHS_MAX + j]; };
  std::memset(B.flags_host, 0, sizeof(int) * n * RHS_MAX);
  batch_put_flags(B);
  batch_replay(B, B.init);
  batch_fetch(B);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < B.nrhs[i]; ++j) {
      bb[base[i] + j] = B.gath_host[(long)(n + i) * RHS_MAX + j];
      if (!std::isfinite(bb[base[i] + j]))
        fail(AMG_ERR_NAN, "instance " + std::to_string(i) + ", right-hand side " + std::to_string(j) +
                              " has non-finite entries");
    }
  int k = 0, it = 0;
  for (;;) {
    int active = 0, cand = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < B.nrhs[i]; ++j) {
        const int q = base[i] + j;
        if (state[q] == 0 && rr(i, j) <= tol * tol * bb[q]) state[q] = 1;
        if (state[q] == 0) ++active;
        if (state[q] == 1) ++cand;
      }
    if ((cand > 0 && active == 0) || k == B.m || (it >= maxiter && cand > 0)) {
      // true residual of every rhs; candidates that pass are done, and the
      // iteration restarts from the true residuals
      batch_replay(B, B.truer);
      batch_fetch(B);
      active = 0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < B.nrhs[i]; ++j) {
          const int q = base[i] + j;
          R.rel[q] = bb[q] > 0 ? std::sqrt(rr(i, j) / bb[q]) : 0.0;
          if (state[q] == 1) {
            if (rr(i, j) <= tol * tol * bb[q]) { state[q] = 2; R.iters[q] = it; }
            else state[q] = 0;
          }
          if (state[q] == 0) ++active;
        }
      k = 0;
    }
    if (active == 0 || it >= maxiter) break;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < B.nrhs[i]; ++j) B.flags_host[(long)i * RHS_MAX + j] = state[base[i] + j] != 0;
    batch_put_flags(B);
    batch_replay(B, B.iters[k]);
    batch_fetch(B);
    ++k;
    ++it;
  }
  if (std::any_of(state.begin(), state.end(), [](int v) { return v == 0; })) {
    batch_replay(B, B.truer);
    batch_fetch(B);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < B.nrhs[i]; ++j) {
        const int q = base[i] + j;
        R.rel[q] = bb[q] > 0 ? std::sqrt(rr(i, j) / bb[q]) : 0.0;
        if (state[q] != 2) R.iters[q] = it;
      }
  }
  R.done.resize(tot);
  for (int q = 0; q < tot; ++q) R.done[q] = (state[q] == 2) || (R.rel[q] <= tol);
  R.outer = it;
  return R;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================


extern "C" {

const char* amg_status_str(amg_status s) {
  switch (s) {
    case AMG_OK: return "ok";
    case AMG_ERR_ARG: return "invalid argument";
    case AMG_ERR_SHAPE: return "shape mismatch";
    case AMG_ERR_NAN: return "non-finite values";
    case AMG_ERR_NOMEM: return "out of device memory";
    case AMG_ERR_HIP: return "HIP runtime error";
    case AMG_ERR_RANK: return "linearly dependent near-null vectors";
    case AMG_ERR_NOCONV: return "not converged";
    case AMG_ERR_STATE: return "invalid state";
    case AMG_ERR_SINGULAR: return "singular coarsest operator";
  }
  return "unknown status";
}

const char* amg_last_error(void) { return last_error().c_str(); }

void amg_default_params(amg_mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nlevels = 2;
  for (int l = 0; l < 3; ++l) {
    for (int mu = 0; mu < 4; ++mu) p->block[l][mu] = 4;
    p->nvec[l] = 8;
  }
  p->nu_pre = 2;
  p->nu_post = 2;
  p->omega = 0.8;
  p->coarse_tol = 0.1;
  p->coarse_maxiter = 64;
  p->coarse_restart = 16;
  p->outer_restart = 16;
  p->inner_prec = AMG_F64;
  p->p_bf16 = 0;
  p->kcycle_tol = 0.1;
  p->kcycle_maxiter = 0;
  p->coarse_dense_max = 4096;
  p->coarse_jacobi = 0;
  p->coarse_eo = 0;
}

amg_status amg_gauge_create(const amg_lattice* lat, const void* dev_links, double mass, void* stream,
                            amg_gauge** out) {
  AMG_TRY
  check_ptr(lat, "lattice");
  check_ptr(dev_links, "links");
  check_ptr(out, "out");
  if (lat->nd != 2 && lat->nd != 4) fail(AMG_ERR_ARG, "nd must be 2 or 4");
  if (!std::isfinite(mass)) fail(AMG_ERR_ARG, "mass must be finite");
  long V = 1;
  for (int mu = 0; mu < lat->nd; ++mu) {
    if (lat->dims[mu] < 2 || lat->dims[mu] % 2) fail(AMG_ERR_SHAPE, "lattice extents must be even and >= 2");
    V *= lat->dims[mu];
  }
  if (V >= (1L << 31)) fail(AMG_ERR_SHAPE, "lattice too large");
  hipStream_t st = as_stream(stream);
  amg_gauge* g = new amg_gauge();
  try {
    g->nd = lat->nd;
    for (int mu = 0; mu < 4; ++mu) g->dims[mu] = mu < lat->nd ? lat->dims[mu] : 1;
    g->V = V;
    g->nc = lat->nd == 2 ? 1 : 3;
    g->ns = lat->nd == 2 ? 2 : 4;
    g->dof = g->nc * g->ns;
    g->mass = mass;
    HIPC(hipGetDevice(&g->device));
    if (g->nd == 2) {
      g->U64.ensure((size_t)2 * V * sizeof(double2));
      g->U32.ensure((size_t)2 * V * sizeof(float2));
      // canonical [mu][site] is the FP64 plane layout; FP32 interleaves (U_1, U_2) per site
      HIPC(hipMemcpyAsync(g->U64.p, dev_links, (size_t)2 * V * sizeof(double2), hipMemcpyDeviceToDevice, st));
      launch_convert<double, float>(g->U32.as<float2>(), (const double2*)dev_links, V, 2, 1, 2, 1, st);
    } else {
      g->U64.ensure((size_t)36 * V * sizeof(double2));
      g->U32.ensure((size_t)36 * V * sizeof(float2));
      launch_links4d_pack(g->U64.as<double2>(), g->U32.as<float2>(), (const double2*)dev_links, V, st);
      // SU(3) links travel as their first two rows (12 reals): a third fewer
      // link bytes and one 16-byte load per element pair in the stencil
      static const bool compress = [] {
        const char* e = std::getenv("AMG_W4_COMPRESS");
        return e ? std::atoi(e) != 0 : true;
      }();
      if (compress) {
        g->Uc64.ensure((size_t)24 * V * sizeof(double2));
        g->Uc32.ensure((size_t)12 * V * sizeof(float4));
        Buf flag;
        flag.ensure(sizeof(int));
        HIPC(hipMemsetAsync(flag.p, 0, sizeof(int), st));
        launch_links4d_compress(g->Uc64.as<double2>(), g->Uc32.as<float4>(), (const double2*)dev_links, V,
                                flag.as<int>(), st);
        int not_su3 = 1;
        HIPC(hipMemcpyAsync(&not_su3, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        g->compressed = not_su3 == 0;
        if (!g->compressed) {
          g->Uc64.release();
          g->Uc32.release();
        }
      }
    }
    g->sc.init(64, RHS_MAX);
    HIPC(hipStreamSynchronize(st));
  } catch (...) {
    delete g;
    throw;
  }
  *out = g;
  AMG_CATCH
}

amg_status amg_gauge_set_mass(amg_gauge* g, double mass) {
  AMG_TRY
  check_ptr(g, "gauge");
  if (!std::isfinite(mass)) fail(AMG_ERR_ARG, "mass must be finite");
  g->mass = mass;
  AMG_CATCH
}

amg_status amg_gauge_info(const amg_gauge* g, int* nd, int* dims4, int* links_compressed) {
  AMG_TRY
  check_ptr(g, "gauge");
  if (nd) *nd = g->nd;
  if (dims4)
    for (int mu = 0; mu < 4; ++mu) dims4[mu] = g->dims[mu];
  if (links_compressed) *links_compressed = g->compressed ? 1 : 0;
  AMG_CATCH
}

amg_status amg_gauge_destroy(amg_gauge* g) {
  AMG_TRY
  delete g;
  AMG_CATCH
}

amg_status amg_apply(const amg_gauge* gc, int dagger, int prec, const void* dev_in, void* dev_out, int nrhs,
                     void* stream) {
  AMG_TRY
  check_ptr(gc, "gauge");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  if (dev_in == dev_out) fail(AMG_ERR_ARG, "in-place application is not supported");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  amg_gauge* g = const_cast<amg_gauge*>(gc);
  hipStream_t st = as_stream(stream);
  const size_t n = (size_t)g->V * g->dof * nrhs;
  const int W = prec == AMG_F64 ? 1 : 2;
  if (prec == AMG_F64) {
    g->tin.ensure(n * sizeof(double2));
    g->tout.ensure(n * sizeof(double2));
    launch_convert<double, double>(g->tin.as<double2>(), (const double2*)dev_in, g->V, g->dof, g->dof, W, nrhs, st);
    wilson_apply<double>(*g, g->mass, dagger, EPI_PLAIN, g->tin.as<double2>(), g->tout.as<double2>(), nullptr, nullptr,
                         nrhs, g->sc.red(0), st);
    launch_convert<double, double>((double2*)dev_out, g->tout.as<double2>(), g->V, g->dof, W, g->dof, nrhs, st);
  } else {
    g->tin.ensure(n * sizeof(float2));
    g->tout.ensure(n * sizeof(float2));
    launch_convert<float, float>(g->tin.as<float2>(), (const float2*)dev_in, g->V, g->dof, g->dof, W, nrhs, st);
    wilson_apply<float>(*g, g->mass, dagger, EPI_PLAIN, g->tin.as<float2>(), g->tout.as<float2>(), nullptr, nullptr,
                        nrhs, g->sc.red(0), st);
    launch_convert<float, float>((float2*)dev_out, g->tout.as<float2>(), g->V, g->dof, W, g->dof, nrhs, st);
  }
  AMG_CATCH
}

}  // extern "C"

// ---- the application of D that allocates nothing ------------------------------
// Staging of the two layout conversions in a fixed device array instead of
// the handle's buffers.  Each GPU that runs the library holds its own copy of
// the array until the process ends; host code reaches it only through the
// per-device address taken with hipGetSymbolAddress (the array's name is a
// host-side stand-in, not a device address).
namespace {
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double2 scratch[kNoallocScratchBytes / sizeof(double2)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (taken once per device,
// with that device current)
void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(AMG_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) fail(AMG_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

amg_status amg_apply_noalloc(const amg_gauge* g, int dagger, int prec, const void* dev_in, void* dev_out, int nrhs,
                             void* stream) {
  AMG_TRY
  check_ptr(g, "gauge");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  if (dev_in == dev_out) fail(AMG_ERR_ARG, "in-place application is not supported");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  const size_t es = prec == AMG_F64 ? sizeof(double2) : sizeof(float2);
  const size_t half = (((size_t)g->V * g->dof * nrhs * es) + 255) & ~size_t(255);
  if (2 * half > kNoallocScratchBytes)
    fail(AMG_ERR_ARG, "amg_apply_noalloc: 2 x V x dof x nrhs complex numbers (" + std::to_string(2 * half) +
                          " bytes) exceed the scratch array of " + std::to_string(kNoallocScratchBytes) + " bytes");
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev != g->device) fail(AMG_ERR_STATE, "the current device is not the gauge handle's device");
  char* base = static_cast<char*>(scratch_ptr(dev));
  hipStream_t st = as_stream(stream);
  const int W = prec == AMG_F64 ? 1 : 2;
  if (prec == AMG_F64) {
    double2* tin = reinterpret_cast<double2*>(base);
    double2* tout = reinterpret_cast<double2*>(base + half);
    launch_convert<double, double>(tin, (const double2*)dev_in, g->V, g->dof, g->dof, W, nrhs, st);
    wilson_apply<double>(*g, g->mass, dagger, EPI_PLAIN, tin, tout, nullptr, nullptr, nrhs, g->sc.red(0), st);
    launch_convert<double, double>((double2*)dev_out, tout, g->V, g->dof, W, g->dof, nrhs, st);
  } else {
    float2* tin = reinterpret_cast<float2*>(base);
    float2* tout = reinterpret_cast<float2*>(base + half);
    launch_convert<float, float>(tin, (const float2*)dev_in, g->V, g->dof, g->dof, W, nrhs, st);
    wilson_apply<float>(*g, g->mass, dagger, EPI_PLAIN, tin, tout, nullptr, nullptr, nrhs, g->sc.red(0), st);
    launch_convert<float, float>((float2*)dev_out, tout, g->V, g->dof, W, g->dof, nrhs, st);
  }
  HIPC(hipGetLastError());
  AMG_CATCH
}

amg_status amg_apply_internal(amg_gauge* g, int dagger, int prec, int nrhs, int iters, void* stream) {
  AMG_TRY
  check_ptr(g, "gauge");
  if (nrhs < 1 || nrhs > RHS_MAX || iters < 0) fail(AMG_ERR_ARG, "bad nrhs / iters");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  hipStream_t st = as_stream(stream);
  const size_t n = (size_t)g->V * g->dof * nrhs;
  const size_t es = prec == AMG_F64 ? sizeof(double2) : sizeof(float2);
  if (g->tin.bytes < n * es) {
    g->tin.ensure(n * es);
    HIPC(hipMemsetAsync(g->tin.p, 0, n * es, st));
  }
  g->tout.ensure(n * es);
  for (int i = 0; i < iters; ++i) {
    if (prec == AMG_F64)
      wilson_apply<double>(*g, g->mass, dagger, EPI_PLAIN, g->tin.as<double2>(), g->tout.as<double2>(), nullptr,
                           nullptr, nrhs, g->sc.red(0), st);
    else
      wilson_apply<float>(*g, g->mass, dagger, EPI_PLAIN, g->tin.as<float2>(), g->tout.as<float2>(), nullptr, nullptr,
                          nrhs, g->sc.red(0), st);
  }
  AMG_CATCH
}

amg_status amg_cgnr_solve(const amg_gauge* gc, const void* dev_chi, void* dev_psi, double tol, int max_iter,
                          amg_solve_info* info, void* stream) {
  AMG_TRY
  check_ptr(gc, "gauge");
  check_ptr(dev_chi, "chi");
  check_ptr(dev_psi, "psi");
  if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_ARG, "bad tol / max_iter");
  amg_gauge* g = const_cast<amg_gauge*>(gc);
  hipStream_t st = as_stream(stream);
  const auto t0 = std::chrono::steady_clock::now();
  const long n = g->V * g->dof;
  for (auto& b : g->cg) b.ensure(n * sizeof(double2));
  double2 *b = g->cg[0].as<double2>(), *x = g->cg[1].as<double2>(), *r = g->cg[2].as<double2>(),
          *s = g->cg[3].as<double2>(), *p = g->cg[4].as<double2>(), *q = g->cg[5].as<double2>();
  enum { SL_BB = 0, SL_RR = 1, SL_QQ = 2, SL_G0 = 3, SL_G1 = 4 };
  launch_convert<double, double>(b, (const double2*)dev_chi, g->V, g->dof, g->dof, 1, 1, st);
  HIPC(hipMemsetAsync(x, 0, n * sizeof(double2), st));
  HIPC(hipMemcpyAsync(r, b, n * sizeof(double2), hipMemcpyDeviceToDevice, st));
  long long nD = 0, nDd = 0;
  wilson_apply<double>(*g, g->mass, 1, EPI_NORM, r, s, nullptr, nullptr, 1, g->sc.red(SL_G0), st);
  nDd++;
  HIPC(hipMemcpyAsync(p, s, n * sizeof(double2), hipMemcpyDeviceToDevice, st));
  launch_norm2<double>(b, n, 1, g->sc.red(SL_BB), st);
  const double bb = g->sc.fetch(SL_BB, 1, st)[0];
  double rr = bb;
  int it = 0, gcur = SL_G0, gnext = SL_G1;
  while (!(rr <= tol * tol * bb) && it < max_iter) {
    wilson_apply<double>(*g, g->mass, 0, EPI_NORM, p, q, nullptr, nullptr, 1, g->sc.red(SL_QQ), st);
    nD++;
    launch_cg_update(x, r, p, q, n, 1, g->sc.red(0), gcur, SL_QQ, SL_RR, st);
    wilson_apply<double>(*g, g->mass, 1, EPI_NORM, r, s, nullptr, nullptr, 1, g->sc.red(gnext), st);
    nDd++;
    launch_cg_pupdate(p, s, n, 1, g->sc.scal.as<double>(), gnext, gcur, st);
    std::swap(gcur, gnext);
    ++it;
    rr = g->sc.fetch(SL_RR, 1, st)[0];
  }
  // true residual
  wilson_apply<double>(*g, g->mass, 0, EPI_RESID, x, r, b, nullptr, 1, g->sc.red(0), st);
  nD++;
  launch_norm2<double>(r, n, 1, g->sc.red(SL_RR), st);
  rr = g->sc.fetch(SL_RR, 1, st)[0];
  launch_convert<double, double>((double2*)dev_psi, x, g->V, g->dof, 1, g->dof, 1, st);
  HIPC(hipStreamSynchronize(st));
  const double rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  if (info) {
    info->iters = it;
    info->converged = rel <= tol;
    info->true_rel_res = rel;
    info->n_fine_D = nD;
    info->n_fine_Ddag = nDd;
    info->n_coarse = 0;
    info->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!(rel <= tol)) fail(AMG_ERR_NOCONV, "CGNR did not reach the tolerance");
  AMG_CATCH
}

amg_status amg_setup(const amg_gauge* g, const amg_mg_params* p, const void* const* dev_nullvecs, void* stream,
                     amg_solver** out) {
  AMG_TRY
  check_ptr(out, "out");
  check_ptr(dev_nullvecs, "nullvecs");
  Solver* S = new_solver(g, p);
  hipStream_t st = as_stream(stream);
  try {
    ensure_work(*S, 1);
    for (int l = 0; l + 1 < (int)S->lv.size(); ++l) {
      check_ptr(dev_nullvecs[l], "nullvecs[l]");
      upload_vectors(*S, l, dev_nullvecs[l], S->lv[l].nv_max, st);
      build_transfer(*S, l, st);
    }
    HIPC(hipStreamSynchronize(st));
  } catch (...) {
    delete S;
    throw;
  }
  *out = S;
  AMG_CATCH
}

amg_status amg_setup_adaptive(const amg_gauge* g, const amg_mg_params* p, const void* const* dev_init, int nu0,
                              int ncyc, void* stream, amg_solver** out) {
  AMG_TRY
  check_ptr(out, "out");
  check_ptr(dev_init, "init");
  if (nu0 < 0 || ncyc < 0) fail(AMG_ERR_ARG, "nu0 / ncyc must be >= 0");
  Solver* S = new_solver(g, p);
  hipStream_t st = as_stream(stream);
  try {
    ensure_work(*S, 1);
    for (int l = 0; l + 1 < (int)S->lv.size(); ++l) {
      check_ptr(dev_init[l], "init[l]");
      adaptive_level(*S, l, dev_init[l], nu0, ncyc, st);
    }
    HIPC(hipStreamSynchronize(st));
  } catch (...) {
    delete S;
    throw;
  }
  *out = S;
  AMG_CATCH
}

amg_status amg_setup_adaptive_levels(const amg_gauge* g, const amg_mg_params* p, const void* const* dev_init,
                                     const int* nu0, const int* ncyc, void* stream, amg_solver** out) {
  AMG_TRY
  check_ptr(out, "out");
  check_ptr(dev_init, "init");
  check_ptr(nu0, "nu0");
  check_ptr(ncyc, "ncyc");
  Solver* S = new_solver(g, p);
  hipStream_t st = as_stream(stream);
  try {
    ensure_work(*S, 1);
    for (int l = 0; l + 1 < (int)S->lv.size(); ++l) {
      check_ptr(dev_init[l], "init[l]");
      if (nu0[l] < 0 || ncyc[l] < 0) fail(AMG_ERR_ARG, "nu0 / ncyc must be >= 0");
      adaptive_level(*S, l, dev_init[l], nu0[l], ncyc[l], st);
    }
    HIPC(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    delete S;
    throw;
  }
  *out = S;
  AMG_CATCH
}

amg_status amg_solver_set_mass(amg_solver* S, double mass) {
  AMG_TRY
  check_ptr(S, "solver");
  if (!std::isfinite(mass)) fail(AMG_ERR_ARG, "mass must be finite");
  const double dm = mass - S->mass;
  S->mass = mass;
  if (dm != 0.0) {
    for (size_t l = 1; l < S->lv.size(); ++l) {
      Level& L = S->lv[l];
      launch_diag_shift(L.Y64.as<double2>(), L.M64.as<double2>(), L.V, L.dof, L.ndir(), dm, nullptr);
      if (S->p.inner_prec == AMG_F32)
        launch_p_convert(L.Y32.p, P_F32, L.Y64.as<double2>(), L.V * L.ndir() * (long)L.dof * L.dof, nullptr);
      if (L.dense) build_dense(*S, (int)l, nullptr);
      if (l + 1 == S->lv.size()) build_jacobi(*S, (int)l, nullptr);  // (solves stop at the last level)
      else L.jac = L.eo = L.s9 = false;
    }
    HIPC(hipStreamSynchronize(nullptr));
  }
  AMG_CATCH
}

amg_status amg_solver_destroy(amg_solver* S) {
  AMG_TRY
  delete S;
  AMG_CATCH
}

amg_status amg_solve(amg_solver* S, const void* dev_chi, void* dev_psi, int nrhs, double tol, int max_iter,
                     amg_solve_info* info, void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_chi, "chi");
  check_ptr(dev_psi, "psi");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_ARG, "bad tol / max_iter");
  hipStream_t st = as_stream(stream);
  const auto t0 = std::chrono::steady_clock::now();
  ensure_work(*S, nrhs);
  const long long d0 = S->nD, dd0 = S->nDd, c0 = S->nC;
  to_internal<double>(*S, 0, (const double2*)dev_chi, S->ob.as<double2>(), nrhs, st);
  OuterResult R = fgcr_outer(*S, S->ob.as<double2>(), S->ox.as<double2>(), nrhs, tol, max_iter, st);
  to_canonical<double>(*S, 0, S->ox.as<double2>(), (double2*)dev_psi, nrhs, st);
  HIPC(hipStreamSynchronize(st));
  check_persistent(*S);
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (int i = 0; i < nrhs; ++i) {
    const bool c = R.rel[i] <= tol;
    all = all && c;
    if (info) {
      info[i].iters = R.iters;
      info[i].converged = c;
      info[i].true_rel_res = R.rel[i];
      info[i].n_fine_D = S->nD - d0;
      info[i].n_fine_Ddag = S->nDd - dd0;
      info[i].n_coarse = S->nC - c0;
      info[i].t_ms = ms;
    }
  }
  if (!all) fail(AMG_ERR_NOCONV, "FGCR did not reach the tolerance");
  AMG_CATCH
}

amg_status amg_get_nullvecs(const amg_solver* S, int level, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_out, "out");
  if (level < 0 || level + 1 >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  const Level& L = S->lv[level];
  to_canonical<double>(*S, level, L.vecs.as<double2>(), (double2*)dev_out, L.nv, as_stream(stream));
  AMG_CATCH
}

amg_status amg_get_coarse_op(const amg_solver* S, int level, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_out, "out");
  if (level < 1 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  const Level& L = S->lv[level];
  // internal blocks are column-major; the ABI exports row-major [t][t']
  launch_block_transpose((double2*)dev_out, L.Y64.as<double2>(), L.V * L.ndir(), L.dof, as_stream(stream));
  AMG_CATCH
}

amg_status amg_set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*, void*),
                             void* ctx) {
  AMG_TRY
  if ((alloc == nullptr) != (release == nullptr)) fail(AMG_ERR_ARG, "give both alloc and release, or neither");
  Allocator& a = allocator();
  a.alloc = alloc;
  a.release = release;
  a.ctx = alloc ? ctx : nullptr;
  AMG_CATCH
}

amg_status amg_level_apply(const amg_solver* Sc, int level, int dagger, int prec, const void* dev_in, void* dev_out,
                           int nrhs, void* stream) {
  AMG_TRY
  check_ptr(Sc, "solver");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  if (dev_in == dev_out) fail(AMG_ERR_ARG, "in-place application is not supported");
  amg_solver* S = const_cast<amg_solver*>(Sc);
  if (level < 0 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  if (prec == AMG_F32 && level > 0 && S->p.inner_prec != AMG_F32) fail(AMG_ERR_STATE, "no FP32 coarse operator");
  hipStream_t st = as_stream(stream);
  ensure_work(*S, nrhs);
  Level& L = S->lv[level];
  if (prec == AMG_F64) {
    double2* a = S->otmp.as<double2>();
    double2* c = L.w64[W_P].as<double2>();
    launch_convert<double, double>(a, (const double2*)dev_in, L.V, L.dof, L.dof, L.lay64.W, nrhs, st);
    op_apply<double>(*S, level, dagger, EPI_PLAIN, a, c, nullptr, nullptr, nrhs, S->sc.red(0), st);
    launch_convert<double, double>((double2*)dev_out, c, L.V, L.dof, L.lay64.W, L.dof, nrhs, st);
  } else {
    // FP64 solvers have no FP32 work vectors on the fine level: size them
    // for this call (no-op when they are large enough already)
    L.w32[W_B].ensure((size_t)L.V * L.dof_max * nrhs * sizeof(float2));
    L.w32[W_P].ensure((size_t)L.V * L.dof_max * nrhs * sizeof(float2));
    float2* a = L.w32[W_B].as<float2>();
    float2* c = L.w32[W_P].as<float2>();
    launch_convert<float, float>(a, (const float2*)dev_in, L.V, L.dof, L.dof, L.lay32.W, nrhs, st);
    op_apply<float>(*S, level, dagger, EPI_PLAIN, a, c, nullptr, nullptr, nrhs, S->sc.red(0), st);
    launch_convert<float, float>((float2*)dev_out, c, L.V, L.dof, L.lay32.W, L.dof, nrhs, st);
  }
  AMG_CATCH
}

amg_status amg_transfer(const amg_solver* Sc, int level, int dir, int prec, const void* dev_in, void* dev_out,
                        int nrhs, void* stream) {
  AMG_TRY
  check_ptr(Sc, "solver");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  amg_solver* S = const_cast<amg_solver*>(Sc);
  if (level < 0 || level + 1 >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  if (dir != 0 && dir != 1) fail(AMG_ERR_ARG, "dir must be 0 (restrict) or 1 (prolong)");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  if (prec == AMG_F32 && S->p.inner_prec != AMG_F32) fail(AMG_ERR_STATE, "no FP32 prolongator");
  hipStream_t st = as_stream(stream);
  ensure_work(*S, nrhs);
  Level& F = S->lv[level];
  if (prec == AMG_F64) {
    const TransferGeom tg = tgeom(*S, level, AMG_F64);
    double2* a = S->otmp.as<double2>();
    if (level > 0) a = F.w64[W_P].as<double2>();
    if (dir == 0) {
      launch_convert<double, double>(a, (const double2*)dev_in, F.V, F.dof, F.dof, F.lay64.W, nrhs, st);
      launch_restrict<double>((double2*)dev_out, a, F.P64.p, P_F64, tg, nrhs, nullptr, st);
    } else {
      launch_prolong<double>(a, (const double2*)dev_in, F.P64.p, P_F64, tg, nrhs, 0, nullptr, st);
      launch_convert<double, double>((double2*)dev_out, a, F.V, F.dof, F.lay64.W, F.dof, nrhs, st);
    }
  } else {
    // the FP32 cycle's transfer: P as the cycle stores it (FP32 or bfloat16)
    const TransferGeom tg = tgeom(*S, level, AMG_F32);
    int pk;
    const void* P = Pstore<float>(*S, level, pk);
    float2* a = F.w32[W_P].as<float2>();
    if (dir == 0) {
      launch_convert<float, float>(a, (const float2*)dev_in, F.V, F.dof, F.dof, F.lay32.W, nrhs, st);
      launch_restrict<float>((float2*)dev_out, a, P, pk, tg, nrhs, nullptr, st);
    } else {
      launch_prolong<float>(a, (const float2*)dev_in, P, pk, tg, nrhs, 0, nullptr, st);
      launch_convert<float, float>((float2*)dev_out, a, F.V, F.dof, F.lay32.W, F.dof, nrhs, st);
    }
  }
  AMG_CATCH
}

amg_status amg_get_prolongator(const amg_solver* Sc, int level, int prec, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(Sc, "solver");
  check_ptr(dev_out, "out");
  amg_solver* S = const_cast<amg_solver*>(Sc);
  if (level < 0 || level + 1 >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  if (prec == AMG_F32 && S->p.inner_prec != AMG_F32) fail(AMG_ERR_STATE, "no FP32 prolongator");
  int pk;
  const void* P = prec == AMG_F64 ? Pstore<double>(*S, level, pk) : Pstore<float>(*S, level, pk);
  launch_p_export((double2*)dev_out, P, pk, tgeom(*S, level, prec), as_stream(stream));
  AMG_CATCH
}

amg_status amg_vcycle(amg_solver* S, const void* dev_b, void* dev_x, int nrhs, void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_b, "b");
  check_ptr(dev_x, "x");
  if (nrhs < 1 || nrhs > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
  hipStream_t st = as_stream(stream);
  ensure_work(*S, nrhs);
  to_internal<double>(*S, 0, (const double2*)dev_b, S->ob.as<double2>(), nrhs, st);
  precondition(*S, S->ob.as<double2>(), S->ox.as<double2>(), nrhs, st);
  to_canonical<double>(*S, 0, S->ox.as<double2>(), (double2*)dev_x, nrhs, st);
  AMG_CATCH
}

amg_status amg_mr(amg_solver* S, int level, int prec, int nu, const void* dev_b, void* dev_x, int nrhs,
                  void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_b, "b");
  check_ptr(dev_x, "x");
  if (level < 0 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  if (nrhs < 1 || nrhs > RHS_MAX || nu < 0) fail(AMG_ERR_ARG, "bad nrhs / nu");
  if (prec != AMG_F64 && prec != AMG_F32) fail(AMG_ERR_ARG, "bad precision");
  if (prec == AMG_F32 && S->p.inner_prec != AMG_F32) fail(AMG_ERR_STATE, "no FP32 operators");
  hipStream_t st = as_stream(stream);
  ensure_work(*S, nrhs);
  Level& L = S->lv[level];
  if (prec == AMG_F64) {
    double2* b = level == 0 ? S->ob.as<double2>() : L.w64[W_B].as<double2>();
    double2* x = level == 0 ? S->ox.as<double2>() : L.w64[W_X].as<double2>();
    launch_convert<double, double>(b, (const double2*)dev_b, L.V, L.dof, L.dof, L.lay64.W, nrhs, st);
    mr_smooth<double>(*S, level, b, x, L.w64[W_R].as<double2>(), L.w64[W_P].as<double2>(), nu, true, true, nrhs, st);
    launch_convert<double, double>((double2*)dev_x, x, L.V, L.dof, L.lay64.W, L.dof, nrhs, st);
  } else {
    float2* b = L.w32[W_B].as<float2>();
    float2* x = L.w32[W_X].as<float2>();
    launch_convert<float, float>(b, (const float2*)dev_b, L.V, L.dof, L.dof, L.lay32.W, nrhs, st);
    mr_smooth<float>(*S, level, b, x, L.w32[W_R].as<float2>(), L.w32[W_P].as<float2>(), nu, true, true, nrhs, st);
    launch_convert<float, float>((float2*)dev_x, x, L.V, L.dof, L.lay32.W, L.dof, nrhs, st);
  }
  AMG_CATCH
}

amg_status amg_profile_enable(amg_solver* S, int kind, int level, int enable) {
  AMG_TRY
  check_ptr(S, "solver");
  if (kind < -1 || kind > 6 || level < -1 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad kind / level");
  S->prof.on = enable != 0;
  S->prof.kind = kind;
  S->prof.level = level;
  S->prof.used = 0;
  AMG_CATCH
}

amg_status amg_profile_read(amg_solver* S, double* total_ms, long long* launches) {
  AMG_TRY
  check_ptr(S, "solver");
  auto& P = S->prof;
  double tot = 0.0;
  if (P.used) HIPC(hipEventSynchronize(P.ev[P.used - 1]));
  for (size_t i = 0; i + 1 < P.used; i += 2) {
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, P.ev[i], P.ev[i + 1]));
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (long long)(P.used / 2);
  AMG_CATCH
}

amg_status amg_profile_read_kind(amg_solver* S, int kind, int level, double* total_ms, long long* launches) {
  AMG_TRY
  check_ptr(S, "solver");
  auto& P = S->prof;
  double tot = 0.0;
  long long n = 0;
  if (P.used) HIPC(hipEventSynchronize(P.ev[P.used - 1]));
  for (size_t i = 0; i + 1 < P.used; i += 2) {
    if (P.tag[i / 2] != ((kind << 8) | level)) continue;
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, P.ev[i], P.ev[i + 1]));
    tot += ms;
    ++n;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  AMG_CATCH
}

amg_status amg_level_info(const amg_solver* S, int level, int* dims4, int* dof, long long* V) {
  AMG_TRY
  check_ptr(S, "solver");
  if (level < 0 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  const Level& L = S->lv[level];
  if (dims4)
    for (int mu = 0; mu < 4; ++mu) dims4[mu] = L.dims[mu];
  if (dof) *dof = L.dof;
  if (V) *V = L.V;
  AMG_CATCH
}

amg_status amg_mg_convergence(amg_solver* S, const void* dev_e0, int iters, double* rho, void* stream) {
  AMG_TRY
  check_ptr(S, "solver");
  check_ptr(dev_e0, "e0");
  check_ptr(rho, "rho");
  if (iters < 1 || iters > 1000) fail(AMG_ERR_ARG, "iters must be 1..1000");
  *rho = mg_convergence(*S, (const double2*)dev_e0, iters, as_stream(stream));
  AMG_CATCH
}

namespace {

// Level 0 from given starting vectors, refined; deeper levels adaptive.
Solver* build_refined(const amg_gauge* g, const amg_mg_params* p, const void* start0, int n_start, int nu_ref,
                      int ncyc_ref, const void* const* dev_init, int nu0, int ncyc, hipStream_t st) {
  Solver* S = new_solver(g, p);
  try {
    ensure_work(*S, 1);
    for (int l = 0; l + 1 < (int)S->lv.size(); ++l) {
      if (l == 0) refined_level(*S, 0, start0, n_start, nu_ref, dev_init[0], ncyc_ref, st);
      else adaptive_level(*S, l, dev_init[l], nu0, ncyc, st);
    }
    HIPC(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipStreamSynchronize(st);
    delete S;
    throw;
  }
  return S;
}

void check_refine_args(const amg_gauge* g, const amg_mg_params* p, const void* const* dev_init, int n_start,
                       int nu_ref, int ncyc_ref, int nu0, int ncyc, amg_solver** out) {
  check_ptr(g, "gauge");
  check_ptr(p, "params");
  check_ptr(dev_init, "init");
  check_ptr(out, "out");
  if (nu_ref < 0 || ncyc_ref < 0 || nu0 < 0 || ncyc < 0) fail(AMG_ERR_ARG, "nu / ncyc must be >= 0");
  if (p->nlevels < 2 || p->nlevels > 4) fail(AMG_ERR_ARG, "nlevels must be 2..4");
  if (n_start < 1 || n_start > p->nvec[0]) fail(AMG_ERR_ARG, "n_start must be 1..nvec[0]");
  if (n_start < p->nvec[0]) check_ptr(dev_init[0], "init[0]");
  for (int l = 1; l + 1 < p->nlevels; ++l) check_ptr(dev_init[l], "init[l]");
}

}  // namespace

amg_status amg_setup_refined(const amg_gauge* g, const amg_mg_params* p, const void* dev_start0, int n_start,
                             int nu_ref, int ncyc_ref, const void* const* dev_init, int nu0, int ncyc, void* stream,
                             amg_solver** out) {
  AMG_TRY
  check_refine_args(g, p, dev_init, n_start, nu_ref, ncyc_ref, nu0, ncyc, out);
  check_ptr(dev_start0, "start vectors");
  *out = build_refined(g, p, dev_start0, n_start, nu_ref, ncyc_ref, dev_init, nu0, ncyc, as_stream(stream));
  AMG_CATCH
}

amg_status amg_setup_learned(const amg_gauge* g, const amg_mg_params* p, amg_cnn* net, const void* const* dev_init,
                             int n_start, int nu_ref, int ncyc_ref, double rho_max, int rho_iters, int nu0, int ncyc,
                             void* stream, amg_solver** out, int* fell_back, double* rho) {
  AMG_TRY
  check_refine_args(g, p, dev_init, n_start, nu_ref, ncyc_ref, nu0, ncyc, out);
  check_ptr(net, "network");
  check_ptr(dev_init[0], "init[0]");
  if (g->nd != 2) fail(AMG_ERR_ARG, "the learned setup is two-dimensional (U(1)) only");
  if (n_start > 8) fail(AMG_ERR_ARG, "the network proposes 8 vectors");
  if (rho_iters < 0 || rho_iters > 1000) fail(AMG_ERR_ARG, "rho_iters must be 0..1000");
  if (rho_iters > 0 && !(rho_max > 0.0)) fail(AMG_ERR_ARG, "rho_max must be positive");
  hipStream_t st = as_stream(stream);
  Solver* S = nullptr;
  double r = -1.0;
  int fb = 0;
  {
    Buf prop;
    prop.ensure((size_t)8 * g->V * 2 * sizeof(double2));
    const amg_status ps = amg_cnn_propose(net, g->U64.p, g->dims[0], g->dims[1], prop.p, stream);
    if (ps != AMG_OK) fail(ps, "amg_cnn_propose: " + last_error());
    try {
      S = build_refined(g, p, prop.p, n_start, nu_ref, ncyc_ref, dev_init, nu0, ncyc, st);
      if (rho_iters > 0) {
        r = mg_convergence(*S, (const double2*)dev_init[0], rho_iters, st);
        if (!(r <= rho_max)) fb = 1;
      }
    } catch (const Fail& f) {
      if (f.s != AMG_ERR_RANK && f.s != AMG_ERR_NAN) {
        delete S;
        throw;
      }
      fb = 1;
    }
  }
  if (fb) {
    delete S;
    S = nullptr;
    S = new_solver(g, p);
    try {
      ensure_work(*S, 1);
      for (int l = 0; l + 1 < (int)S->lv.size(); ++l) adaptive_level(*S, l, dev_init[l], nu0, ncyc, st);
      HIPC(hipStreamSynchronize(st));
      if (rho_iters > 0) r = mg_convergence(*S, (const double2*)dev_init[0], rho_iters, st);
    } catch (...) {
      (void)hipStreamSynchronize(st);
      delete S;
      throw;
    }
  }
  if (fell_back) *fell_back = fb;
  if (rho) *rho = r;
  *out = S;
  AMG_CATCH
}

amg_status amg_batch_create(amg_solver* const* solvers, const int* nrhs, int n, int autotune, void* stream,
                            amg_batch** out) {
  AMG_TRY
  check_ptr(solvers, "solvers");
  check_ptr(nrhs, "nrhs");
  check_ptr(out, "out");
  if (n < 1 || n > 4096) fail(AMG_ERR_ARG, "batch size must be 1..4096");
  Batch* B = new Batch();
  try {
    B->n = n;
    HIPC(hipStreamCreateWithFlags(&B->st, hipStreamNonBlocking));
    HIPC(hipStreamSynchronize(as_stream(stream)));
    const Solver* s0 = solvers[0];
    check_ptr(s0, "solvers[0]");
    for (int i = 0; i < n; ++i) {
      Solver* S = solvers[i];
      check_ptr(S, "solvers[i]");
      if (S->g->nd != 2) fail(AMG_ERR_ARG, "batched solves support the 2d operator");
      if (S->lv.size() != s0->lv.size() || S->p.inner_prec != s0->p.inner_prec || S->p.p_bf16 != s0->p.p_bf16 ||
          S->p.nu_pre != s0->p.nu_pre || S->p.nu_post != s0->p.nu_post || S->p.outer_restart != s0->p.outer_restart ||
          S->p.coarse_maxiter != s0->p.coarse_maxiter || S->p.coarse_restart != s0->p.coarse_restart ||
          S->p.kcycle_maxiter != s0->p.kcycle_maxiter)
        fail(AMG_ERR_ARG, "batched solvers must share the hierarchy depth and solver parameters");
      for (size_t l = 0; l < S->lv.size(); ++l)
        if (S->lv[l].dof != s0->lv[l].dof) fail(AMG_ERR_ARG, "batched solvers must share the dof per level");
      if (nrhs[i] < 1 || nrhs[i] > RHS_MAX) fail(AMG_ERR_ARG, "bad nrhs");
      for (int j = 0; j < i; ++j)
        if (solvers[j] == S) fail(AMG_ERR_ARG, "a solver appears twice in the batch");
      B->S.push_back(S);
      B->nrhs.push_back(nrhs[i]);
      ensure_work(*S, nrhs[i]);
    }
    B->m = s0->p.outer_restart;
    B->flags_dev.ensure(sizeof(int) * n * RHS_MAX);
    HIPC(hipMemset(B->flags_dev.p, 0, sizeof(int) * n * RHS_MAX));
    B->gath_dev.ensure(sizeof(double) * 2 * n * RHS_MAX);
    HIPC(hipHostMalloc((void**)&B->gath_host, sizeof(double) * 2 * n * RHS_MAX, hipHostMallocDefault));
    HIPC(hipHostMalloc((void**)&B->flags_host, sizeof(int) * n * RHS_MAX, hipHostMallocDefault));
    for (int i = 0; i < n; ++i) B->S[i]->outer_flags = B->flags_dev.as<int>() + (long)i * RHS_MAX;
    // one kernel choice for every instance at a stage: the multi-rhs coarse
    // kernel for all of them (any nrhs) or for none
    std::vector<int> saved_mrhs(n);
    for (int i = 0; i < n; ++i) {
      saved_mrhs[i] = B->S[i]->mrhs_min;
      // the coarsest level by GCR on every instance: an exact (dense) solve on
      // some instances and GCR on others would not merge stage by stage
      B->S[i]->no_dense = true;
    }
    auto set_mrhs = [&](int on) {
      for (int i = 0; i < n; ++i) B->S[i]->mrhs_min = on ? 1 : (1 << 30);
    };
    const int saved = red_block_cap();
    if (autotune) {
      // autotune the launch shapes jointly: the grid of the reducing kernels
      // x the coarse stencil (multi-rhs MFMA kernel or one rhs per grid row);
      // each candidate is built and one outer iteration (the first direction)
      // timed on a unit source, three replays after one warm-up
      for (int i = 0; i < n; ++i) {
        Solver& S = *B->S[i];
        const long cnt = S.lv[0].per_rhs() * B->nrhs[i];
        std::vector<double2> ones(cnt, make_double2(1.0, 0.0));
        HIPC(hipMemcpy(S.ob.p, ones.data(), sizeof(double2) * cnt, hipMemcpyHostToDevice));
      }
      float best = 1e30f;
      hipEvent_t e0, e1;
      HIPC(hipEventCreate(&e0));
      HIPC(hipEventCreate(&e1));
      for (int mr : {1, 0})
        for (int cap : {128, 256, 512, 1024}) {
          set_mrhs(mr);
          set_red_block_cap(cap);
          batch_build(*B);
          batch_replay(*B, B->init);
          batch_replay(*B, B->iters[0]);
          HIPC(hipEventRecord(e0, B->st));
          for (int rep = 0; rep < 3; ++rep) batch_replay(*B, B->iters[0]);
          HIPC(hipEventRecord(e1, B->st));
          HIPC(hipEventSynchronize(e1));
          float ms = 0.f;
          HIPC(hipEventElapsedTime(&ms, e0, e1));
          B->trials.push_back({cap, mr, ms / 3.f});
          if (ms < best) {
            best = ms;
            B->red_cap = cap;
            B->mrhs = mr;
          }
          auto drop = [](Batch::Seg& g) { if (g.exec) (void)hipGraphExecDestroy(g.exec); g.exec = nullptr; };
          drop(B->init);
          drop(B->truer);
          for (auto& g : B->iters) drop(g);
        }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    } else if (const char* e = std::getenv("AMG_BATCH_MRHS")) {
      B->mrhs = std::atoi(e) != 0 ? 1 : 0;
    }
    set_mrhs(B->mrhs);
    set_red_block_cap(B->red_cap);
    batch_build(*B);
    set_red_block_cap(saved);
    for (int i = 0; i < n; ++i) {
      B->S[i]->outer_flags = nullptr;
      B->S[i]->mrhs_min = saved_mrhs[i];
      B->S[i]->no_dense = false;
    }
    HIPC(hipStreamSynchronize(B->st));
  } catch (...) {
    delete B;
    throw;
  }
  *out = B;
  AMG_CATCH
}

amg_status amg_batch_solve(amg_batch* B, const void* const* dev_chi, void* const* dev_psi, double tol, int max_iter,
                           amg_solve_info* info, void* stream) {
  AMG_TRY
  check_ptr(B, "batch");
  check_ptr(dev_chi, "chi");
  check_ptr(dev_psi, "psi");
  if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_ARG, "bad tol / max_iter");
  const auto t0 = std::chrono::steady_clock::now();
  HIPC(hipStreamSynchronize(as_stream(stream)));
  for (int i = 0; i < B->n; ++i) {
    check_ptr(dev_chi[i], "chi[i]");
    check_ptr(dev_psi[i], "psi[i]");
    to_internal<double>(*B->S[i], 0, (const double2*)dev_chi[i], B->S[i]->ob.as<double2>(), B->nrhs[i], B->st);
  }
  BatchResult R = batch_run(*B, tol, max_iter);
  for (int i = 0; i < B->n; ++i)
    to_canonical<double>(*B->S[i], 0, B->S[i]->ox.as<double2>(), (double2*)dev_psi[i], B->nrhs[i], B->st);
  HIPC(hipStreamSynchronize(B->st));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (size_t q = 0; q < R.rel.size(); ++q) {
    all = all && R.done[q];
    if (info) {
      info[q].iters = R.iters[q];
      info[q].converged = R.done[q];
      info[q].true_rel_res = R.rel[q];
      info[q].n_fine_D = info[q].n_fine_Ddag = info[q].n_coarse = 0;
      info[q].t_ms = ms;
    }
  }
  if (!all) fail(AMG_ERR_NOCONV, "batched FGCR did not reach the tolerance for every right-hand side");
  AMG_CATCH
}

amg_status amg_batch_info(const amg_batch* B, int* red_cap, int* stages_per_iteration) {
  AMG_TRY
  check_ptr(B, "batch");
  if (red_cap) *red_cap = B->red_cap;
  if (stages_per_iteration) *stages_per_iteration = B->iters.empty() ? 0 : (int)B->iters[0].ops.size();
  AMG_CATCH
}

int amg_batch_tuning(const amg_batch* B, int max, int* red_cap, int* mrhs, float* ms_per_iteration) {
  if (!B) return -1;
  const int n = (int)B->trials.size();
  for (int i = 0; i < n && i < max; ++i) {
    if (red_cap) red_cap[i] = B->trials[i].red_cap;
    if (mrhs) mrhs[i] = B->trials[i].mrhs;
    if (ms_per_iteration) ms_per_iteration[i] = B->trials[i].ms;
  }
  return n;
}

amg_status amg_batch_info2(const amg_batch* B, int* red_cap, int* mrhs, int* stages_per_iteration) {
  AMG_TRY
  check_ptr(B, "batch");
  if (red_cap) *red_cap = B->red_cap;
  if (mrhs) *mrhs = B->mrhs;
  if (stages_per_iteration) *stages_per_iteration = B->iters.empty() ? 0 : (int)B->iters[0].ops.size();
  AMG_CATCH
}

amg_status amg_batch_destroy(amg_batch* B) {
  AMG_TRY
  delete B;
  AMG_CATCH
}

}  // extern "C"

// Host runtime of the multigrid for the normal equations A = D^dag D on 2d
// lattices (the paper's own variant, numerical-test section): the hierarchy
// from given or adaptive near-null vectors, Galerkin products and the
// smoothed prolongator by probing, the V-cycle of the five steps before
// Eq. (3) with the frozen two-step smoother, and CG / MG-CG.  Every
// arithmetic step runs in the library's gfx950 kernels; the host sequences
// launches and reads a few scalars (step lengths and norms during set-up, one
// residual norm per CG iteration).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "amg.h"
#include "gauge.h"
#include "hostutil.h"
#include "kernels.h"

using namespace amg;
using namespace amg::host;

namespace {

constexpr int PROBE_CHUNK = 64;     // probe vectors per batch of launches
constexpr int NRM_MMAX = 16;        // largest M
constexpr long EXPORT_MAX = 1L << 28;

// scalar slots
enum {
  S_DOT = 0,    // dot3: 3 slots
  S_PQ = 4,     // <p, A p>: 3 slots
  S_G0 = 8,     // rho, two alternating dot3 results: 3 slots each
  S_G1 = 12,
  S_RR = 16,    // |r|^2 after a CG update
  S_BB = 17,    // |b|^2
  S_TT = 18,    // |b - A x|^2
  S_NSLOTS = 32
};

struct NLevel {
  int d1 = 0, d2 = 0;
  long V = 0;
  int dof = 0;
  Layout lay{};
  long n() const { return V * dof; }
  // coarsening to the level below (all but the coarsest)
  int b1 = 0, b2 = 0, M = 0;
  NGeom g{};
  Buf vecs;                 // near-null vectors [M][n], internal layout
  Buf sb;                   // smoother / power start vector
  Buf Pt, Psa;              // tentative and smoothed prolongator
  double tau0 = 0.0, tau1 = 0.0, lambda = 0.0, sa_omega = 0.0;
  // operator (levels >= 1) and exact solve
  Buf Y;
  bool dense = false;
  Buf Ainv;
  // level 0: A = D^dag D also stored as a 9-point box stencil (2 x 2 blocks),
  // applied in one launch instead of D then D^dag
  bool box = false;
  // work
  Buf b, x, r, t, u, r2;
  Buf cr, cz, cp, cq, ct;   // CG on this level
  const double2* P() const { return g.sa ? Psa.as<double2>() : Pt.as<double2>(); }
};

}  // namespace

struct amg_normal {
  amg_gauge* g = nullptr;
  amg_normal_params p{};
  double mass = 0.0;
  std::vector<NLevel> lv;
  Scratch sc;
  Buf tD;                    // fine-level D output (up to PROBE_CHUNK right-hand sides)
  Buf pe, px, py, pz;        // probe buffers
  Buf gjA, gjB, gjkey, gjint;
  Buf err;
  Buf cgflag;                // batched CG: stop flag and performed-iteration counter
  Buf io;                    // internal copies of fine fields at the C ABI
  long long nD = 0, nDd = 0;
};

namespace {

using Normal = amg_normal;

void check_ptr(const void* p, const char* what) {
  if (p == nullptr) fail(AMG_ERR_ARG, std::string(what) + " is NULL");
}

int period(int c, int pmin) {
  for (int p = pmin; p <= c; ++p)
    if (c % p == 0) return p;
  return 0;
}

double fetch1(Normal& S, int slot, hipStream_t st) { return S.sc.fetch(slot, 1, st)[0]; }

BoxArgs box_args(const NLevel& L, int epi) {
  BoxArgs a;
  a.Y = L.Y.as<double2>();
  a.L1 = L.d1;
  a.L2 = L.d2;
  a.M = L.dof;
  a.lay = L.lay;
  a.epi = epi;
  return a;
}

// the box stencil of level l (level 0 only when built) with an epilogue;
// level 0 counts as one D and one D^dag application per field
void box_apply(Normal& S, int l, BoxArgs a, int nrhs, hipStream_t st) {
  launch_box(a, nrhs, st);
  if (l == 0 && !a.stop) {
    S.nD += nrhs;
    S.nDd += nrhs;
  }
}

bool stencil_level(const Normal& S, int l) { return l > 0 || S.lv[0].box; }

// out = A_l in (epi 0) or out = b - A_l in (epi 1), nrhs fields.  stop: the
// launches do nothing while *stop != 0 (the caller then counts the fine
// applications that ran itself)
void apply_A(Normal& S, int l, const double2* in, double2* out, const double2* b, int epi, int nrhs, hipStream_t st,
             const int* stop = nullptr) {
  NLevel& L = S.lv[l];
  if (!stencil_level(S, l)) {
    S.tD.ensure((size_t)L.n() * nrhs * sizeof(double2));
    wilson_apply<double>(*S.g, S.mass, 0, EPI_PLAIN, in, S.tD.as<double2>(), nullptr, nullptr, nrhs,
                         S.sc.red(0, stop), st);
    wilson_apply<double>(*S.g, S.mass, 1, epi ? EPI_RESID : EPI_PLAIN, S.tD.as<double2>(), out, b, nullptr, nrhs,
                         S.sc.red(0, stop), st);
    if (!stop) {
      S.nD += nrhs;
      S.nDd += nrhs;
    }
  } else {
    BoxArgs a = box_args(L, epi ? BOX_RESID : BOX_APPLY);
    a.in = in;
    a.out = out;
    a.b = b;
    a.stop = stop;
    box_apply(S, l, a, nrhs, st);
  }
}

void dot3(Normal& S, const double2* a, const double2* b, long n, int slot, hipStream_t st) {
  launch_dot3(a, b, n, S.sc.red(slot), st);
}

void ensure_level_work(NLevel& L) {
  const size_t nb = (size_t)L.n() * sizeof(double2);
  for (Buf* b : {&L.b, &L.x, &L.r, &L.t, &L.u, &L.r2, &L.cr, &L.cz, &L.cp, &L.cq, &L.ct}) b->ensure(nb);
}

// ---- set-up pieces ----------------------------------------------------------------

// Rayleigh quotient of A_l after power_steps steps p <- A p / |A p| from sb
double power_lmax(Normal& S, int l, hipStream_t st) {
  NLevel& L = S.lv[l];
  const long n = L.n();
  double2 *p = L.x.as<double2>(), *q = L.t.as<double2>();
  dot3(S, L.sb.as<double2>(), L.sb.as<double2>(), n, S_DOT, st);
  launch_scale_norm(p, L.sb.as<double2>(), S.sc.scal.as<double>(), S_DOT, n, st);
  for (int k = 0; k < S.p.power_steps; ++k) {
    apply_A(S, l, p, q, nullptr, 0, 1, st);
    dot3(S, q, q, n, S_DOT, st);
    launch_scale_norm(p, q, S.sc.scal.as<double>(), S_DOT, n, st);
  }
  apply_A(S, l, p, q, nullptr, 0, 1, st);
  dot3(S, p, q, n, S_DOT, st);
  return fetch1(S, S_DOT, st);
}

// frozen step lengths: two MR steps on A_l x = sb from x = 0
void frozen_steps(Normal& S, int l, hipStream_t st) {
  NLevel& L = S.lv[l];
  const long n = L.n();
  double2 *r = L.r.as<double2>(), *t = L.t.as<double2>();
  launch_fill<double>(r, L.sb.as<double2>(), n, 1, st);
  double tau[2];
  for (int i = 0; i < 2; ++i) {
    apply_A(S, l, r, t, nullptr, 0, 1, st);
    dot3(S, t, r, n, S_DOT, st);
    const double* h = S.sc.fetch(S_DOT, 3, st);
    if (!(h[2] > 0.0)) fail(AMG_ERR_STATE, "frozen smoother: A r = 0 on level " + std::to_string(l));
    tau[i] = S.p.omega * h[0] / h[2];
    launch_axpy3(r, r, t, -tau[i], n, st);
  }
  L.tau0 = tau[0];
  L.tau1 = tau[1];
}

// smoothed P of coarsening l: (1 - omega A_l) P_tent column by column, from
// probes of period >= 2 (the widened blocks of one colour are disjoint)
void build_psa(Normal& S, int l, hipStream_t st) {
  NLevel& F = S.lv[l];
  const NGeom& g = F.g;
  NGeom gt = g;
  gt.sa = 0;
  F.lambda = power_lmax(S, l, st);
  if (!(F.lambda > 0.0)) fail(AMG_ERR_STATE, "power estimate of A is not positive");
  F.sa_omega = S.p.sa_factor / F.lambda;
  const int q1 = period(g.c1, 2), q2 = period(g.c2, 2);
  const int np = q1 * q2 * g.M;
  const long n = F.n(), nc = (long)g.c1 * g.c2 * g.M;
  F.Psa.ensure((size_t)n * 4 * g.M * sizeof(double2));
  S.pe.ensure((size_t)nc * PROBE_CHUNK * sizeof(double2));
  S.px.ensure((size_t)n * PROBE_CHUNK * sizeof(double2));
  S.py.ensure((size_t)n * PROBE_CHUNK * sizeof(double2));
  for (int q0 = 0; q0 < np; q0 += PROBE_CHUNK) {
    const int nq = std::min(PROBE_CHUNK, np - q0);
    launch_probe(S.pe.as<double2>(), g.c1, g.c2, g.M, q1, q2, q0, nq, st);
    launch_normal_prolong(S.px.as<double2>(), S.pe.as<double2>(), F.Pt.as<double2>(), gt, nq, 0, st);
    apply_A(S, l, S.px.as<double2>(), S.py.as<double2>(), nullptr, 0, nq, st);
    launch_axpy3(S.py.as<double2>(), S.px.as<double2>(), S.py.as<double2>(), -F.sa_omega, n * nq, st);
    launch_psa_scatter(F.Psa.as<double2>(), S.py.as<double2>(), g, q1, q2, q0, nq, st);
  }
}

// A_{l+1} = P^dag A_l P as a box stencil, from probes of period >= 3
void galerkin(Normal& S, int l, hipStream_t st) {
  NLevel& F = S.lv[l];
  NLevel& C = S.lv[l + 1];
  const NGeom& g = F.g;
  const int p1 = period(g.c1, 3), p2 = period(g.c2, 3);
  const int np = p1 * p2 * g.M;
  const long n = F.n(), nc = (long)g.c1 * g.c2 * g.M;
  C.Y.ensure((size_t)C.V * 9 * g.M * g.M * sizeof(double2));
  S.pe.ensure((size_t)nc * PROBE_CHUNK * sizeof(double2));
  S.px.ensure((size_t)n * PROBE_CHUNK * sizeof(double2));
  S.py.ensure((size_t)n * PROBE_CHUNK * sizeof(double2));
  S.pz.ensure((size_t)nc * PROBE_CHUNK * sizeof(double2));
  for (int q0 = 0; q0 < np; q0 += PROBE_CHUNK) {
    const int nq = std::min(PROBE_CHUNK, np - q0);
    launch_probe(S.pe.as<double2>(), g.c1, g.c2, g.M, p1, p2, q0, nq, st);
    launch_normal_prolong(S.px.as<double2>(), S.pe.as<double2>(), F.P(), g, nq, 0, st);
    apply_A(S, l, S.px.as<double2>(), S.py.as<double2>(), nullptr, 0, nq, st);
    launch_normal_restrict(S.pz.as<double2>(), S.py.as<double2>(), F.P(), g, nq, st);
    launch_galerkin_box_scatter(C.Y.as<double2>(), S.pz.as<double2>(), g.c1, g.c2, g.M, p1, p2, q0, nq, st);
  }
}

// A_0 = D^dag D as a box stencil of 2 x 2 blocks, by probing the two Wilson
// applications with coloured unit vectors (period >= 3), on lattices up to
// 2^18 sites (beyond, the two stencil launches move fewer bytes than the
// 576-byte box blocks per site)
constexpr long FINE_BOX_MAX_SITES = 1L << 18;
void build_fine_box(Normal& S, hipStream_t st) {
  NLevel& L = S.lv[0];
  L.box = false;
  const int p1 = period(L.d1, 3), p2 = period(L.d2, 3);
  if (!S.p.fine_box || L.V > FINE_BOX_MAX_SITES || p1 == 0 || p2 == 0) return;
  const int np = p1 * p2 * 2;
  const long n = L.n();
  L.Y.ensure((size_t)L.V * 9 * 4 * sizeof(double2));
  for (Buf* b : {&S.pe, &S.px, &S.py, &S.pz, &S.tD}) b->ensure((size_t)n * PROBE_CHUNK * sizeof(double2));
  for (int q0 = 0; q0 < np; q0 += PROBE_CHUNK) {
    const int nq = std::min(PROBE_CHUNK, np - q0);
    launch_probe(S.pe.as<double2>(), L.d1, L.d2, 2, p1, p2, q0, nq, st);                       // [site][spin]
    launch_convert<double, double>(S.px.as<double2>(), S.pe.as<double2>(), L.V, 2, 2, 1, nq, st);  // -> planes
    wilson_apply<double>(*S.g, S.mass, 0, EPI_PLAIN, S.px.as<double2>(), S.tD.as<double2>(), nullptr, nullptr, nq,
                         S.sc.red(0), st);
    wilson_apply<double>(*S.g, S.mass, 1, EPI_PLAIN, S.tD.as<double2>(), S.py.as<double2>(), nullptr, nullptr, nq,
                         S.sc.red(0), st);
    launch_convert<double, double>(S.pz.as<double2>(), S.py.as<double2>(), L.V, 2, 1, 2, nq, st);  // -> [site][spin]
    launch_galerkin_box_scatter(L.Y.as<double2>(), S.pz.as<double2>(), L.d1, L.d2, 2, p1, p2, q0, nq, st);
  }
  L.box = true;
}

// P and A_{l+1} of coarsening l from its first M vectors
void build_coarsening(Normal& S, int l, int M, hipStream_t st) {
  NLevel& F = S.lv[l];
  NLevel& C = S.lv[l + 1];
  F.g = NGeom{F.d1, F.d2, F.b1, F.b2, C.d1, C.d2, F.dof, M, S.p.sa_factor > 0.0 ? 1 : 0, F.lay};
  C.dof = M;
  C.lay = Layout{C.V, M, M};
  ensure_level_work(C);
  if (normal_orth_lds(F.g) > 64 * 1024) fail(AMG_ERR_SHAPE, "block too large for the orthonormalisation (64 KiB LDS)");
  F.Pt.ensure((size_t)F.n() * M * sizeof(double2));
  HIPC(hipMemsetAsync(S.err.p, 0, sizeof(int), st));
  NGeom gt = F.g;
  gt.sa = 0;
  launch_normal_orth(F.Pt.as<double2>(), F.vecs.as<double2>(), gt, F.n(), S.err.as<int>(), st);
  int herr = 0;
  HIPC(hipMemcpyAsync(&herr, S.err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (herr) fail(AMG_ERR_RANK, "near-null vectors of coarsening " + std::to_string(l) + " are dependent on a block");
  if (F.g.sa) build_psa(S, l, st);
  else F.lambda = F.sa_omega = 0.0;
  galerkin(S, l, st);
}

// dense inverse of level l's box stencil
void build_dense(Normal& S, int l, hipStream_t st) {
  NLevel& L = S.lv[l];
  const long N = L.n();
  L.dense = false;
  const size_t nn = (size_t)N * N;
  S.gjA.ensure(nn * sizeof(double2));
  S.gjB.ensure(nn * sizeof(double2));
  S.gjkey.ensure((size_t)(N + 2) * sizeof(unsigned long long));
  S.gjint.ensure((size_t)(3 * N + 8) * sizeof(int));
  L.Ainv.ensure(nn * sizeof(double2));
  int* piv = S.gjint.as<int>();
  int* used = piv + N;
  int* pinv = used + N;
  int* err = pinv + N;
  HIPC(hipMemsetAsync(S.gjA.p, 0, nn * sizeof(double2), st));
  launch_box_dense(S.gjA.as<double2>(), L.Y.as<double2>(), L.d1, L.d2, L.dof, st);
  launch_gj_invert(S.gjA.as<double2>(), S.gjB.as<double2>(), N, S.gjkey.as<unsigned long long>(), piv, used, pinv, err,
                   L.Ainv.as<double2>(), nullptr, st);
  int herr = 0;
  HIPC(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (herr) fail(AMG_ERR_SINGULAR, "the operator of level " + std::to_string(l) + " is singular");
  L.dense = true;
}

// ---- solve pieces ------------------------------------------------------------------

struct CgOut {
  int iters = 0, restarts = 0;
  bool converged = false;
  double rel = INFINITY;
};

CgOut cg_solve(Normal& S, int l, const double2* b, double2* x, double tol, int maxiter, int lstop, hipStream_t st);

// (stop: a batched CG's flag, only with a dense coarse level)
void coarse_solve(Normal& S, int l, const double2* b, double2* x, hipStream_t st, const int* stop) {
  NLevel& L = S.lv[l];
  if (L.dense) launch_dense_apply<double>(x, b, L.Ainv.as<double2>(), L.n(), 1, stop, st);
  else if (stop) fail(AMG_ERR_STATE, "a batched CG needs an exact coarsest solve");
  else cg_solve(S, l, b, x, S.p.setup_coarse_tol, S.p.setup_coarse_maxiter, -1, st);
}

// x = V b on level l, recursion down to level lstop (solved exactly); with
// stop, every launch does nothing while *stop != 0 and nothing is counted
void vcycle(Normal& S, int l, int lstop, const double2* b, double2* x, hipStream_t st, const int* stop = nullptr) {
  if (l == lstop) {
    coarse_solve(S, l, b, x, st, stop);
    return;
  }
  NLevel& F = S.lv[l];
  NLevel& C = S.lv[l + 1];
  const long n = F.n();
  double2 *r = F.r.as<double2>(), *t = F.t.as<double2>();
  if (stencil_level(S, l)) {
    // the same five steps with the smoother's updates in the stencil's epilogue
    BoxArgs a = box_args(F, BOX_SMOOTH0);
    a.stop = stop;
    a.in = b;                                // 1. x = tau0 b, r = b - tau0 A b
    a.out = r;
    a.x = x;
    a.c1 = F.tau0;
    box_apply(S, l, a, 1, st);
    a.epi = BOX_SMOOTH1;                     //    x += tau1 r, r2 = r - tau1 A r
    a.in = r;
    a.out = F.r2.as<double2>();
    a.c1 = F.tau1;
    box_apply(S, l, a, 1, st);
    launch_normal_restrict(C.b.as<double2>(), F.r2.as<double2>(), F.P(), F.g, 1, st, stop);   // 2.-3.
    vcycle(S, l + 1, lstop, C.b.as<double2>(), C.x.as<double2>(), st, stop);
    launch_normal_prolong(x, C.x.as<double2>(), F.P(), F.g, 1, 1, st, stop);                  // 4.
    a.epi = BOX_RESID;                       // 5. r = b - A x, then x += R r
    a.in = x;
    a.b = b;
    a.out = r;
    a.x = nullptr;
    box_apply(S, l, a, 1, st);
    a.epi = BOX_POST;
    a.in = r;
    a.out = nullptr;
    a.x = x;
    a.c1 = F.tau0 + F.tau1;
    a.c2 = F.tau0 * F.tau1;
    box_apply(S, l, a, 1, st);
    return;
  }
  // 1. x = R^dag b: the two frozen steps from x = 0 (R = R^dag)
  apply_A(S, l, b, t, nullptr, 0, 1, st, stop);
  launch_smooth_step(x, r, b, t, F.tau0, n, 1, st, stop);
  apply_A(S, l, r, t, nullptr, 0, 1, st, stop);
  launch_smooth_step(x, r, nullptr, t, F.tau1, n, 0, st, stop);
  // 2.-3. restrict the residual, cycle below
  launch_normal_restrict(C.b.as<double2>(), r, F.P(), F.g, 1, st, stop);
  vcycle(S, l + 1, lstop, C.b.as<double2>(), C.x.as<double2>(), st, stop);
  // 4. coarse-grid correction
  launch_normal_prolong(x, C.x.as<double2>(), F.P(), F.g, 1, 1, st, stop);
  // 5. x += R (b - A x)
  apply_A(S, l, x, r, b, 1, 1, st, stop);
  apply_A(S, l, r, t, nullptr, 0, 1, st, stop);
  launch_smooth_post(x, r, t, F.tau0 + F.tau1, F.tau0 * F.tau1, n, st, stop);
}

// CG on A_l x = b from x = 0; lstop >= 0: preconditioned by one V-cycle to lstop
CgOut cg_solve(Normal& S, int l, const double2* b, double2* x, double tol, int maxiter, int lstop, hipStream_t st) {
  NLevel& L = S.lv[l];
  const long n = L.n();
  double2 *r = L.cr.as<double2>(), *p = L.cp.as<double2>(), *q = L.cq.as<double2>(), *t = L.ct.as<double2>();
  double2* z = lstop >= 0 ? L.cz.as<double2>() : r;
  double* scal = S.sc.scal.as<double>();
  CgOut o;
  launch_fill<double>(x, nullptr, n, 1, st);
  launch_fill<double>(r, b, n, 1, st);
  launch_norm2<double>(b, n, 1, S.sc.red(S_BB), st);
  const double bb = fetch1(S, S_BB, st);
  if (!(bb > 0.0)) {
    o.converged = true;
    o.rel = 0.0;
    return o;
  }
  const double tol2 = tol * tol * bb;
  double rr = bb;
  int gcur = S_G0, gnext = S_G1;
  bool fresh = true;
  // Steps are enqueued in batches with no host round trip: the update's last
  // block raises a device stop flag once the recursive residual is below
  // tol, after which the rest of the batch does nothing, so the iterates and
  // the count are those of the step-by-step loop; the host then confirms the
  // residual by recomputing it (else restarts from it).
  const int batch = lstop >= 0 ? 8 : 16;
  const int per_step = lstop >= 0 ? 5 : 1;  // fine applications per step (outer + V-cycle's four)
  S.cgflag.ensure(4 * sizeof(int));
  int* stop = S.cgflag.as<int>();
  int* cnt = stop + 1;
  HIPC(hipMemsetAsync(stop, 0, 2 * sizeof(int), st));
  int* hflags = reinterpret_cast<int*>(S.sc.host + 2 * RHS_MAX);
  int counted = 0;
  // plain CG: rho = <r, r> is the |r|^2 the update reduces anyway; it goes
  // into the slot that becomes the next step's rho
  const bool plain = lstop < 0;
  if (plain) launch_norm2<double>(r, n, 1, S.sc.red(gnext), st);
  while (o.iters < maxiter) {
    if (rr <= tol2) {
      apply_A(S, l, x, t, b, 1, 1, st);
      launch_norm2<double>(t, n, 1, S.sc.red(S_TT), st);
      const double tt = fetch1(S, S_TT, st);
      if (tt <= tol2) {
        o.converged = true;
        break;
      }
      launch_fill<double>(r, t, n, 1, st);
      if (plain) launch_norm2<double>(r, n, 1, S.sc.red(gnext), st);
      HIPC(hipMemsetAsync(stop, 0, sizeof(int), st));
      rr = tt;
      fresh = true;
      ++o.restarts;
    }
    const int K = std::min(batch, maxiter - o.iters);
    for (int k = 0; k < K; ++k) {
      if (!plain) {
        vcycle(S, l, lstop, r, z, st, stop);
        launch_dot3(r, z, n, S.sc.red(gnext), st, stop);          // rho = Re <r, z>
      }
      launch_cgb_dir(p, z, n, scal, gnext, gcur, fresh ? 1 : 0, stop, st);
      apply_A(S, l, p, q, nullptr, 0, 1, st, stop);
      launch_dot3(p, q, n, S.sc.red(S_PQ), st, stop);
      launch_cgb_update(x, r, p, q, n, S.sc.red(0), gnext, S_PQ, S_RR, plain ? gcur : -1, tol2, stop, cnt, st);
      std::swap(gcur, gnext);
      fresh = false;
    }
    HIPC(hipMemcpyAsync(hflags, stop, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    rr = fetch1(S, S_RR, st);  // (synchronises the stream)
    o.iters = hflags[1];
    if (l == 0) {  // fine applications of the steps that ran
      S.nD += (long long)per_step * (o.iters - counted);
      S.nDd += (long long)per_step * (o.iters - counted);
    }
    counted = o.iters;
  }
  apply_A(S, l, x, t, b, 1, 1, st);
  launch_norm2<double>(t, n, 1, S.sc.red(S_TT), st);
  o.rel = std::sqrt(fetch1(S, S_TT, st) / bb);
  o.converged = o.rel <= tol;
  return o;
}

// ---- construction --------------------------------------------------------------------

void check_params(const amg_gauge* g, const amg_normal_params* p) {
  if (g->nd != 2) fail(AMG_ERR_SHAPE, "the normal-equation multigrid is for 2d lattices");
  if (p->nlevels < 2 || p->nlevels > 4) fail(AMG_ERR_ARG, "nlevels must be 2..4");
  if (!(p->omega > 0.0) || !(p->sa_factor >= 0.0) || p->power_steps < 0) fail(AMG_ERR_ARG, "bad omega / sa_factor");
  if (p->coarse_dense_max < 1 || p->coarse_dense_max > AMG_DENSE_MAX) fail(AMG_ERR_ARG, "bad coarse_dense_max");
  if (!(p->setup_coarse_tol > 0.0) || p->setup_coarse_maxiter < 1 || p->setup_dense_max < 0 ||
      p->setup_dense_max > AMG_DENSE_MAX)
    fail(AMG_ERR_ARG, "bad setup coarse solve");
  int d1 = g->dims[0], d2 = g->dims[1];
  for (int l = 0; l + 1 < p->nlevels; ++l) {
    const int b1 = p->block[l][0], b2 = p->block[l][1], M = p->nvec[l];
    if (b1 < 1 || b2 < 1 || d1 % b1 || d2 % b2) fail(AMG_ERR_SHAPE, "blocks must divide the extents");
    if (M < 1 || M > NRM_MMAX) fail(AMG_ERR_ARG, "nvec must be 1..16");
    const int dof = l == 0 ? 2 : p->nvec[l - 1];
    if (b1 * b2 * dof < M) fail(AMG_ERR_SHAPE, "more vectors than block components");
    d1 /= b1;
    d2 /= b2;
    if (period(d1, 3) == 0 || period(d2, 3) == 0)
      fail(AMG_ERR_SHAPE, "coarse extents must have a divisor >= 3 (box-stencil probing)");
    if (p->sa_factor > 0.0 && (b1 < 3 || b2 < 3 || period(d1, 2) == 0 || period(d2, 2) == 0))
      fail(AMG_ERR_SHAPE, "smoothed P needs blocks >= 3");
  }
  if ((long)d1 * d2 * p->nvec[p->nlevels - 2] > p->coarse_dense_max)
    fail(AMG_ERR_ARG, "the coarsest level exceeds coarse_dense_max (it is solved exactly)");
}

Normal* new_normal(const amg_gauge* g, const amg_normal_params* p) {
  check_ptr(g, "gauge");
  check_ptr(p, "params");
  check_params(g, p);
  Normal* S = new Normal;
  S->g = const_cast<amg_gauge*>(g);
  S->p = *p;
  S->mass = g->mass;
  S->sc.init(S_NSLOTS, 8);
  S->err.ensure(sizeof(int) * 4);
  S->lv.resize(p->nlevels);
  int d1 = g->dims[0], d2 = g->dims[1];
  for (int l = 0; l < p->nlevels; ++l) {
    NLevel& L = S->lv[l];
    L.d1 = d1;
    L.d2 = d2;
    L.V = (long)d1 * d2;
    if (l == 0) {
      L.dof = 2;
      L.lay = Layout{L.V, 2, 1};
      ensure_level_work(L);
    }
    if (l + 1 < p->nlevels) {
      L.b1 = p->block[l][0];
      L.b2 = p->block[l][1];
      L.M = p->nvec[l];
      d1 /= L.b1;
      d2 /= L.b2;
    }
  }
  return S;
}

// canonical [k][V][dof] -> internal layout of level l (k fields)
void to_internal(Normal& S, int l, const double2* canon, double2* out, int k, hipStream_t st) {
  const NLevel& L = S.lv[l];
  launch_convert<double, double>(out, canon, L.V, L.dof, L.dof, L.lay.W, k, st);
}
void to_canonical(Normal& S, int l, const double2* in, double2* canon, int k, hipStream_t st) {
  const NLevel& L = S.lv[l];
  launch_convert<double, double>(canon, in, L.V, L.dof, L.lay.W, L.dof, k, st);
}

void upload_level_inputs(Normal& S, int l, const void* vecs, const void* sb, hipStream_t st) {
  NLevel& L = S.lv[l];
  check_ptr(vecs, "vectors");
  check_ptr(sb, "smoother vector");
  L.vecs.ensure((size_t)L.n() * L.M * sizeof(double2));
  L.sb.ensure((size_t)L.n() * sizeof(double2));
  to_internal(S, l, (const double2*)vecs, L.vecs.as<double2>(), L.M, st);
  to_internal(S, l, (const double2*)sb, L.sb.as<double2>(), 1, st);
}

void finish(Normal& S, hipStream_t st) {
  const int nl = (int)S.lv.size();
  for (int l = 0; l + 1 < nl; ++l) frozen_steps(S, l, st);
  build_dense(S, nl - 1, st);
  HIPC(hipStreamSynchronize(st));
}

void adaptive_coarsening(Normal& S, int l, int nu0, int ncyc, hipStream_t st) {
  NLevel& F = S.lv[l];
  NLevel& C = S.lv[l + 1];
  const long n = F.n();
  double2* v0 = F.vecs.as<double2>();
  frozen_steps(S, l, st);
  // vector 0: nu0 MR steps on A v = 0 (Eq. (4))
  {
    double2 *r = F.r.as<double2>(), *t = F.t.as<double2>();
    apply_A(S, l, v0, t, nullptr, 0, 1, st);
    launch_axpy3(r, t, t, -2.0, n, st);   // r = -A v
    for (int i = 0; i < nu0; ++i) {
      apply_A(S, l, r, t, nullptr, 0, 1, st);
      dot3(S, t, r, n, S_DOT, st);
      launch_mr_step(v0, r, t, S.sc.scal.as<double>(), S_DOT, S.p.omega, n, st);
    }
  }
  for (int k = 1; k < F.M; ++k) {
    build_coarsening(S, l, k, st);
    C.dense = false;
    if (C.n() <= S.p.setup_dense_max) build_dense(S, l + 1, st);
    double2* e = v0 + (long)k * n;
    for (int c = 0; c < ncyc; ++c) {
      apply_A(S, l, e, F.u.as<double2>(), nullptr, 0, 1, st);
      vcycle(S, l, l + 1, F.u.as<double2>(), F.x.as<double2>(), st);
      launch_axpy3(e, e, F.x.as<double2>(), -1.0, n, st);
    }
    dot3(S, e, e, n, S_DOT, st);
    launch_scale_norm(e, e, S.sc.scal.as<double>(), S_DOT, n, st);
  }
  build_coarsening(S, l, F.M, st);
  C.dense = false;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

void amg_normal_default_params(amg_normal_params* p) {
  if (!p) return;
  *p = amg_normal_params{};
  p->nlevels = 3;
  for (int l = 0; l < 3; ++l) {
    p->block[l][0] = p->block[l][1] = 4;
    p->nvec[l] = 8;
  }
  p->omega = 0.8;
  p->sa_factor = 4.0 / 3.0;
  p->power_steps = 20;
  p->coarse_dense_max = 4096;
  p->fine_box = 1;
  p->setup_dense_max = 1024;
  p->setup_coarse_tol = 1e-6;
  p->setup_coarse_maxiter = 20000;
}

amg_status amg_normal_setup(const amg_gauge* g, const amg_normal_params* p, const void* const* dev_vecs,
                            const void* const* dev_sb, void* stream, amg_normal** out) {
  AMG_TRY
  check_ptr(out, "out");
  check_ptr(dev_vecs, "vectors");
  check_ptr(dev_sb, "smoother vectors");
  Normal* S = new_normal(g, p);
  hipStream_t st = as_stream(stream);
  try {
    const int nl = (int)S->lv.size();
    build_fine_box(*S, st);
    for (int l = 0; l + 1 < nl; ++l) {
      upload_level_inputs(*S, l, dev_vecs[l], dev_sb[l], st);
      build_coarsening(*S, l, S->lv[l].M, st);
    }
    finish(*S, st);
  } catch (...) {
    delete S;
    throw;
  }
  *out = S;
  AMG_CATCH
}

amg_status amg_normal_setup_adaptive(const amg_gauge* g, const amg_normal_params* p, const void* const* dev_init,
                                     const void* const* dev_sb, const int* nu0, const int* ncyc, void* stream,
                                     amg_normal** out) {
  AMG_TRY
  check_ptr(out, "out");
  check_ptr(dev_init, "init");
  check_ptr(dev_sb, "smoother vectors");
  check_ptr(nu0, "nu0");
  check_ptr(ncyc, "ncyc");
  Normal* S = new_normal(g, p);
  hipStream_t st = as_stream(stream);
  try {
    const int nl = (int)S->lv.size();
    build_fine_box(*S, st);
    for (int l = 0; l + 1 < nl; ++l) {
      if (nu0[l] < 0 || ncyc[l] < 0) fail(AMG_ERR_ARG, "negative nu0 / ncyc");
      upload_level_inputs(*S, l, dev_init[l], dev_sb[l], st);
      adaptive_coarsening(*S, l, nu0[l], ncyc[l], st);
    }
    finish(*S, st);
  } catch (...) {
    delete S;
    throw;
  }
  *out = S;
  AMG_CATCH
}

amg_status amg_normal_set_mass(amg_normal* S, double mass, void* stream) {
  AMG_TRY
  check_ptr(S, "handle");
  if (!std::isfinite(mass)) fail(AMG_ERR_ARG, "mass must be finite");
  hipStream_t st = as_stream(stream);
  S->mass = mass;
  const int nl = (int)S->lv.size();
  build_fine_box(*S, st);
  for (int l = 0; l + 1 < nl; ++l) build_coarsening(*S, l, S->lv[l].M, st);
  finish(*S, st);
  AMG_CATCH
}

amg_status amg_normal_solve(amg_normal* S, const void* dev_chi, void* dev_psi, double tol, int max_iter,
                            int precond, amg_normal_info* info, void* stream) {
  AMG_TRY
  check_ptr(S, "handle");
  check_ptr(dev_chi, "chi");
  check_ptr(dev_psi, "psi");
  if (!(tol > 0.0) || max_iter < 0 || (precond != 0 && precond != 1)) fail(AMG_ERR_ARG, "bad tol / max_iter / precond");
  hipStream_t st = as_stream(stream);
  const auto t0 = std::chrono::steady_clock::now();
  S->nD = S->nDd = 0;
  NLevel& L = S->lv[0];
  const long n = L.n();
  S->io.ensure((size_t)4 * n * sizeof(double2));
  double2 *chi = S->io.as<double2>(), *b = chi + n, *x = b + n, *t = x + n;
  to_internal(*S, 0, (const double2*)dev_chi, chi, 1, st);
  wilson_apply<double>(*S->g, S->mass, 1, EPI_PLAIN, chi, b, nullptr, nullptr, 1, S->sc.red(0), st);
  S->nDd++;
  const CgOut o = cg_solve(*S, 0, b, x, tol, max_iter, precond ? (int)S->lv.size() - 1 : -1, st);
  to_canonical(*S, 0, x, (double2*)dev_psi, 1, st);
  // |chi - D psi| / |chi|
  wilson_apply<double>(*S->g, S->mass, 0, EPI_RESID, x, t, chi, nullptr, 1, S->sc.red(0), st);
  S->nD++;
  launch_norm2<double>(t, n, 1, S->sc.red(S_TT), st);
  launch_norm2<double>(chi, n, 1, S->sc.red(S_BB), st);
  const double* h = S->sc.fetch(S_BB, 2, st);
  const double relD = h[0] > 0.0 ? std::sqrt(h[1] / h[0]) : 0.0;
  if (info) {
    info->iters = o.iters;
    info->converged = o.converged;
    info->restarts = o.restarts;
    info->rel_res_normal = o.rel;
    info->rel_res_D = relD;
    info->n_fine_D = S->nD;
    info->n_fine_Ddag = S->nDd;
    info->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!o.converged) fail(AMG_ERR_NOCONV, "CG did not reach the tolerance");
  AMG_CATCH
}

amg_status amg_normal_vcycle(amg_normal* S, const void* dev_in, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(S, "handle");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  hipStream_t st = as_stream(stream);
  const long n = S->lv[0].n();
  S->io.ensure((size_t)4 * n * sizeof(double2));
  double2 *in = S->io.as<double2>(), *out = in + n;
  to_internal(*S, 0, (const double2*)dev_in, in, 1, st);
  vcycle(*S, 0, (int)S->lv.size() - 1, in, out, st);
  to_canonical(*S, 0, out, (double2*)dev_out, 1, st);
  HIPC(hipStreamSynchronize(st));
  AMG_CATCH
}

amg_status amg_normal_level_apply(amg_normal* S, int level, const void* dev_in, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(S, "handle");
  check_ptr(dev_in, "in");
  check_ptr(dev_out, "out");
  if (level < 0 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  hipStream_t st = as_stream(stream);
  const long n = S->lv[level].n();
  if (level == 0) {
    S->io.ensure((size_t)4 * n * sizeof(double2));
    double2 *in = S->io.as<double2>(), *out = in + n;
    to_internal(*S, 0, (const double2*)dev_in, in, 1, st);
    apply_A(*S, 0, in, out, nullptr, 0, 1, st);
    to_canonical(*S, 0, out, (double2*)dev_out, 1, st);
  } else {
    apply_A(*S, level, (const double2*)dev_in, (double2*)dev_out, nullptr, 0, 1, st);
  }
  HIPC(hipStreamSynchronize(st));
  AMG_CATCH
}

amg_status amg_normal_export(amg_normal* S, int level, int what, void* dev_out, void* stream) {
  AMG_TRY
  check_ptr(S, "handle");
  check_ptr(dev_out, "out");
  const int nl = (int)S->lv.size();
  hipStream_t st = as_stream(stream);
  if (what == 0 || what == 2) {
    if (level < 0 || level + 1 >= nl) fail(AMG_ERR_ARG, "bad coarsening");
    const NLevel& F = S->lv[level];
    const NLevel& C = S->lv[level + 1];
    if (what == 0) {
      const long rows = F.n(), cols = C.n();
      if (rows * cols > EXPORT_MAX) fail(AMG_ERR_ARG, "prolongator too large to export densely");
      HIPC(hipMemsetAsync(dev_out, 0, (size_t)rows * cols * sizeof(double2), st));
      launch_normal_p_dense((double2*)dev_out, F.P(), F.g, st);
    } else {
      to_canonical(*S, level, F.vecs.as<double2>(), (double2*)dev_out, F.M, st);
    }
  } else if (what == 1) {
    if (level < 1 || level >= nl) fail(AMG_ERR_ARG, "bad level");
    const NLevel& L = S->lv[level];
    const long N = L.n();
    if (N * N > EXPORT_MAX) fail(AMG_ERR_ARG, "operator too large to export densely");
    HIPC(hipMemsetAsync(dev_out, 0, (size_t)N * N * sizeof(double2), st));
    launch_box_dense((double2*)dev_out, L.Y.as<double2>(), L.d1, L.d2, L.dof, st);
  } else {
    fail(AMG_ERR_ARG, "bad export kind");
  }
  HIPC(hipStreamSynchronize(st));
  AMG_CATCH
}

amg_status amg_normal_level_info(const amg_normal* S, int level, int* dims2, int* dof, double* taus2,
                                 double* lambda_omega2) {
  AMG_TRY
  check_ptr(S, "handle");
  if (level < 0 || level >= (int)S->lv.size()) fail(AMG_ERR_ARG, "bad level");
  const NLevel& L = S->lv[level];
  if (dims2) {
    dims2[0] = L.d1;
    dims2[1] = L.d2;
  }
  if (dof) *dof = L.dof;
  if (taus2) {
    taus2[0] = L.tau0;
    taus2[1] = L.tau1;
  }
  if (lambda_omega2) {
    lambda_omega2[0] = L.lambda;
    lambda_omega2[1] = L.sa_omega;
  }
  AMG_CATCH
}

amg_status amg_normal_destroy(amg_normal* S) {
  AMG_TRY
  delete S;
  AMG_CATCH
}

}  // extern "C"

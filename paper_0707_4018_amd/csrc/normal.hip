// Kernels of the multigrid for the normal equations A = D^dag D on 2d
// lattices (the paper's own variant, numerical-test section):
//   * block orthonormalisation of M near-null vectors without chiral split
//     (Eq. (5) and the text after it), the tentative prolongator;
//   * prolongation / restriction with the tentative P (one coarse site per
//     fine site) or the smoothed P = (1 - omega A) P_tent, whose column of
//     block J lives on J widened by one site (D^dag D and every Galerkin
//     operator built from it couple a site only to its 3 x 3 box), so a fine
//     site meets at most 2 x 2 blocks;
//   * the coarse operators as 9-point box stencils of M x M blocks, their
//     Galerkin products by probing with coloured unit vectors, and the dense
//     matrix of the coarsest one;
//   * the frozen two-step smoother, minimal-residual updates and the dot
//     products they need.
// All arithmetic in FP64.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "kernels.h"

namespace amg {
namespace {

#define GRID_STRIDE(i, n) \
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

inline unsigned nblk(long n, long cap = 1L << 16) {
  long b = (n + 255) / 256;
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

constexpr int NRM_MMAX = 16;  // largest number of vectors per coarsening

__device__ __forceinline__ int wrapc(int x, int L) { return x < 0 ? x + L : (x >= L ? x - L : x); }

// Coarse coordinate of slot a (0: lower, 1: upper candidate) of fine
// coordinate x along one axis, and whether the slot's block reaches x.
// Tentative P: one candidate, the block holding x.  Smoothed P: the blocks
// whose widened range [b J - 1, b J + b] holds x: J = x / b (or x / b - 1 at
// the block's first site, x / b + 1 at its last).
__device__ __forceinline__ int slot_coord(int x, int b, int c, int sa, int a, bool& valid) {
  if (!sa) {
    valid = true;
    return x / b;
  }
  const int t = x % b;
  const int hi = x / b + (t == b - 1 ? 1 : 0);
  valid = a == 1 || t == 0 || t == b - 1;
  return wrapc(a ? hi : hi - 1, c);
}

// ---- block orthonormalisation (tentative P) ----------------------------------
// One wave per coarse site J.  The block's rows (site, component) are spread
// over the lanes (row = lane + 64 i); the M vectors restricted to the block
// sit in LDS as W[row][k].  Modified Gram-Schmidt applied twice in vector
// order, then normalisation; a vector whose remainder falls below 1e-10 of
// its original norm sets *err (rank deficiency).
__global__ __launch_bounds__(64) void orth_kernel(double2* __restrict__ P, const double2* __restrict__ vecs, NGeom g,
                                                  long vstride, int* err) {
  extern __shared__ double2 W[];
  const int J = blockIdx.x;
  const int lane = threadIdx.x;
  const int J1 = J % g.c1, J2 = J / g.c1;
  const int bs = g.b1 * g.b2, R = bs * g.dof, M = g.M;
  gptr<const double2> v = gl(vecs);
  auto site_of = [&](int row) -> long {
    const int i = row / g.dof;
    const int x1 = J1 * g.b1 + i % g.b1, x2 = J2 * g.b2 + i / g.b1;
    return (long)x2 * g.f1 + x1;
  };
  for (int row = lane; row < R; row += 64) {
    const long s = site_of(row);
    const int d = row % g.dof;
    for (int k = 0; k < M; ++k) W[row * M + k] = v[k * vstride + g.lf.off(s, d)];
  }
  for (int k = 0; k < M; ++k) {
    double w0 = 0.0;
    for (int row = lane; row < R; row += 64) {
      const double2 w = W[row * M + k];
      w0 += w.x * w.x + w.y * w.y;
    }
    w0 = sqrt(wave_sum(w0));
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < k; ++i) {
        double re = 0.0, im = 0.0;  // <q_i, w>
        for (int row = lane; row < R; row += 64) {
          const double2 q = W[row * M + i], w = W[row * M + k];
          re += q.x * w.x + q.y * w.y;
          im += q.x * w.y - q.y * w.x;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        for (int row = lane; row < R; row += 64) {
          const double2 q = W[row * M + i];
          double2 w = W[row * M + k];
          w.x -= re * q.x - im * q.y;
          w.y -= re * q.y + im * q.x;
          W[row * M + k] = w;
        }
      }
    double nr = 0.0;
    for (int row = lane; row < R; row += 64) {
      const double2 w = W[row * M + k];
      nr += w.x * w.x + w.y * w.y;
    }
    nr = sqrt(wave_sum(nr));
    if (!(nr > 1e-10 * w0) || w0 == 0.0) {
      if (lane == 0) atomicOr(err, 1);
      nr = 1.0;
    }
    const double inv = 1.0 / nr;
    for (int row = lane; row < R; row += 64) {
      double2 w = W[row * M + k];
      w.x *= inv;
      w.y *= inv;
      W[row * M + k] = w;
    }
  }
  gptr<double2> out = gl(P);
  for (int row = lane; row < R; row += 64) {
    const long s = site_of(row);
    const int d = row % g.dof;
    for (int k = 0; k < M; ++k) out[(s * g.dof + d) * (long)M + k] = W[row * M + k];
  }
}

// ---- transfers ----------------------------------------------------------------
// P row (s, d) slot q, column k: P[((s dof + d) NS + q) M + k], NS = 1
// (tentative) or 4 (smoothed, slots (a1, a2) = q & 1, q >> 1).
// out (fine, layout lf) = [out +] P in (coarse, [J][k])
__global__ __launch_bounds__(256) void prolong_kernel(double2* __restrict__ out, const double2* __restrict__ in,
                                                      const double2* __restrict__ P, NGeom g, int accumulate,
                                                      const int* stop) {
  if (stop && *gl(stop)) return;
  const int rhs = blockIdx.y;
  const int NS = g.sa ? 4 : 1, M = g.M;
  const long Vf = (long)g.f1 * g.f2, Vc = (long)g.c1 * g.c2;
  gptr<double2> o = gl(out) + (long)rhs * Vf * g.dof;
  gptr<const double2> c = gl(in) + (long)rhs * Vc * M;
  gptr<const double2> p = gl(P);
  GRID_STRIDE(i, Vf * g.dof) {
    const long s = i / g.dof;
    const int d = (int)(i % g.dof);
    const int x1 = (int)(s % g.f1), x2 = (int)(s / g.f1);
    double2 acc = make_double2(0.0, 0.0);
    for (int q = 0; q < NS; ++q) {
      bool v1, v2;
      const int J1 = slot_coord(x1, g.b1, g.c1, g.sa, q & 1, v1);
      const int J2 = slot_coord(x2, g.b2, g.c2, g.sa, q >> 1, v2);
      if (!(v1 && v2)) continue;
      gptr<const double2> row = p + ((s * g.dof + d) * NS + q) * (long)M;
      gptr<const double2> cj = c + ((long)J2 * g.c1 + J1) * M;
      for (int k = 0; k < M; ++k) cfma<double>(acc, row[k], cj[k]);
    }
    const long off = g.lf.off(s, d);
    if (accumulate) {
      const double2 y = o[off];
      acc.x += y.x;
      acc.y += y.y;
    }
    o[off] = acc;
  }
}

// out (coarse, [J][k]) = P^dag in (fine, layout lf).  One wave per coarse
// site J: the rows (site, component) of J's support (the block, widened by
// one site for the smoothed P) are spread over the lanes, each lane keeps the
// M partial sums, and M wave sums finish them.
__global__ __launch_bounds__(256) void restrict_kernel(double2* __restrict__ out, const double2* __restrict__ in,
                                                       const double2* __restrict__ P, NGeom g, const int* stop) {
  if (stop && *gl(stop)) return;
  const int rhs = blockIdx.y;
  const int NS = g.sa ? 4 : 1, M = g.M, w = g.sa ? 1 : 0;
  const long Vf = (long)g.f1 * g.f2, Vc = (long)g.c1 * g.c2;
  const long J = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (J >= Vc) return;  // uniform per wave
  gptr<double2> o = gl(out) + (long)rhs * Vc * M;
  gptr<const double2> f = gl(in) + (long)rhs * Vf * g.dof;
  gptr<const double2> p = gl(P);
  const int J1 = (int)(J % g.c1), J2 = (int)(J / g.c1);
  const int e1 = g.b1 + 2 * w, e2 = g.b2 + 2 * w;
  const int rows = e1 * e2 * g.dof;
  double2 acc[NRM_MMAX];
#pragma unroll
  for (int k = 0; k < NRM_MMAX; ++k) acc[k] = make_double2(0.0, 0.0);
  for (int row = lane; row < rows; row += 64) {
    const int d = row % g.dof;
    const int u = row / g.dof;
    const int x1 = wrapc(J1 * g.b1 + u % e1 - w, g.f1), x2 = wrapc(J2 * g.b2 + u / e1 - w, g.f2);
    int q = 0;
    if (g.sa) {
      bool v;
      q = (slot_coord(x1, g.b1, g.c1, 1, 1, v) == J1 ? 1 : 0) + 2 * (slot_coord(x2, g.b2, g.c2, 1, 1, v) == J2 ? 1 : 0);
    }
    const long s = (long)x2 * g.f1 + x1;
    const double2 fv = f[g.lf.off(s, d)];
    gptr<const double2> pr = p + ((s * g.dof + d) * NS + q) * (long)M;
#pragma unroll
    for (int k = 0; k < NRM_MMAX; ++k)
      if (k < M) cjfma<double>(acc[k], pr[k], fv);
  }
#pragma unroll
  for (int k = 0; k < NRM_MMAX; ++k) {
    if (k < M) {
      const double re = wave_sum(acc[k].x), im = wave_sum(acc[k].y);
      if (lane == 0) o[J * M + k] = make_double2(re, im);
    }
  }
}

// ---- 9-point box stencil ------------------------------------------------------
// Y[((j 9 + dir) M + c) M + r], dir = (d1 + 1) + 3 (d2 + 1): the M x M block
// coupling row r of site j to column c of site j + (d1, d2).  Fields in any
// Layout (fine planes or coarse [site][k]).  With y = Y in, the epilogue is
//   BOX_APPLY   out = y
//   BOX_RESID   out = b - y
//   BOX_SMOOTH0 x = c1 in, out = in - c1 y              (first frozen step, in = b)
//   BOX_SMOOTH1 x += c1 in, out = in - c1 y             (next step; out must not alias in)
//   BOX_POST    x += c1 in - c2 y                       (x += R r with R = c1 - c2 A)
__device__ __forceinline__ void box_epilogue(const BoxArgs& a, long ro, long off, double2 y) {
  switch (a.epi) {
    case BOX_APPLY: gl(a.out)[ro + off] = y; break;
    case BOX_RESID: {
      const double2 bv = gl(a.b)[ro + off];
      gl(a.out)[ro + off] = make_double2(bv.x - y.x, bv.y - y.y);
      break;
    }
    case BOX_SMOOTH0:
    case BOX_SMOOTH1: {
      const double2 v = gl(a.in)[ro + off];
      double2 xv = a.epi == BOX_SMOOTH0 ? make_double2(0.0, 0.0) : gl(a.x)[ro + off];
      xv.x += a.c1 * v.x;
      xv.y += a.c1 * v.y;
      gl(a.x)[ro + off] = xv;
      gl(a.out)[ro + off] = make_double2(v.x - a.c1 * y.x, v.y - a.c1 * y.y);
      break;
    }
    default: {  // BOX_POST
      const double2 v = gl(a.in)[ro + off];
      double2 xv = gl(a.x)[ro + off];
      xv.x += a.c1 * v.x - a.c2 * y.x;
      xv.y += a.c1 * v.y - a.c2 * y.y;
      gl(a.x)[ro + off] = xv;
    }
  }
}

// one thread per (site, row)
__global__ __launch_bounds__(256) void box_kernel(BoxArgs a) {
  if (a.stop && *gl(a.stop)) return;
  const int rhs = blockIdx.y;
  const int M = a.M, L1 = a.L1, L2 = a.L2;
  const long V = (long)L1 * L2, n = V * M, ro = rhs * a.lay.per_rhs();
  gptr<const double2> x = gl(a.in) + ro;
  gptr<const double2> y = gl(a.Y);
  GRID_STRIDE(i, n) {
    const long j = i / M;
    const int r = (int)(i % M);
    const int j1 = (int)(j % L1), j2 = (int)(j / L1);
    double2 acc = make_double2(0.0, 0.0);
    for (int d2 = -1; d2 <= 1; ++d2) {
      const int n2 = wrapc(j2 + d2, L2);
      for (int d1 = -1; d1 <= 1; ++d1) {
        const long nb = (long)n2 * L1 + wrapc(j1 + d1, L1);
        const int dir = (d1 + 1) + 3 * (d2 + 1);
        gptr<const double2> blk = y + (j * 9 + dir) * (long)M * M + r;
        for (int c = 0; c < M; ++c) cfma<double>(acc, blk[(long)c * M], x[a.lay.off(nb, c)]);
      }
    }
    box_epilogue(a, ro, a.lay.off(j, r), acc);
  }
}

// M = 2 (the fine D^dag D): one thread per site computes both rows, so the
// nine neighbours' two components are loaded once
__global__ __launch_bounds__(256) void box2_kernel(BoxArgs a) {
  if (a.stop && *gl(a.stop)) return;
  const int rhs = blockIdx.y;
  const int L1 = a.L1, L2 = a.L2;
  const long V = (long)L1 * L2, ro = rhs * a.lay.per_rhs();
  gptr<const double2> x = gl(a.in) + ro;
  gptr<const double2> y = gl(a.Y);
  GRID_STRIDE(j, V) {
    const int j1 = (int)(j % L1), j2 = (int)(j / L1);
    double2 acc0 = make_double2(0.0, 0.0), acc1 = make_double2(0.0, 0.0);
#pragma unroll
    for (int dir = 0; dir < 9; ++dir) {
      const int d1 = dir % 3 - 1, d2 = dir / 3 - 1;
      const long nb = (long)wrapc(j2 + d2, L2) * L1 + wrapc(j1 + d1, L1);
      const double2 v0 = x[a.lay.off(nb, 0)], v1 = x[a.lay.off(nb, 1)];
      gptr<const double2> blk = y + (j * 9 + dir) * 4;  // [col][row]
      cfma<double>(acc0, blk[0], v0);
      cfma<double>(acc0, blk[2], v1);
      cfma<double>(acc1, blk[1], v0);
      cfma<double>(acc1, blk[3], v1);
    }
    box_epilogue(a, ro, a.lay.off(j, 0), acc0);
    box_epilogue(a, ro, a.lay.off(j, 1), acc1);
  }
}

// The same for 3 <= M <= 8 with one wave per site: lane l = c M + r (l < M^2)
// takes column c of row r in all nine directions (each direction's block is
// one contiguous read of M^2 entries), and the M partial sums of a row are
// added through LDS.
__global__ __launch_bounds__(256) void box_wave_kernel(BoxArgs a) {
  __shared__ double2 part[4][64];
  if (a.stop && *gl(a.stop)) return;  // uniform: the whole launch returns
  const int rhs = blockIdx.y;
  const int M = a.M, L1 = a.L1, L2 = a.L2;
  const long V = (long)L1 * L2, ro = rhs * a.lay.per_rhs();
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long j = (long)blockIdx.x * 4 + wv;
  const bool site = j < V;
  const int c = lane / M, r = lane - c * M;
  double2 acc = make_double2(0.0, 0.0);
  if (site && lane < M * M) {
    gptr<const double2> x = gl(a.in) + ro;
    gptr<const double2> y = gl(a.Y) + j * 9 * (long)M * M + lane;
    const int j1 = (int)(j % L1), j2 = (int)(j / L1);
#pragma unroll
    for (int dir = 0; dir < 9; ++dir) {
      const int d1 = dir % 3 - 1, d2 = dir / 3 - 1;
      const long nb = (long)wrapc(j2 + d2, L2) * L1 + wrapc(j1 + d1, L1);
      cfma<double>(acc, y[(long)dir * M * M], x[a.lay.off(nb, c)]);
    }
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (site && lane < M) {
    double2 sum = make_double2(0.0, 0.0);
    for (int cc = 0; cc < M; ++cc) {
      const double2 t = part[wv][cc * M + lane];
      sum.x += t.x;
      sum.y += t.y;
    }
    box_epilogue(a, ro, a.lay.off(j, lane), sum);
  }
}

// dense[(j M + r) N + (J M + c)] = Y block (j, dir)[c][r], J = j + dir
// (extents >= 3: the nine neighbours are distinct sites); dense zeroed before
__global__ __launch_bounds__(256) void box_dense_kernel(double2* __restrict__ A, const double2* __restrict__ Y, int L1,
                                                        int L2, int M) {
  const long V = (long)L1 * L2, N = V * M;
  GRID_STRIDE(i, V * 9 * M * M) {
    const int r = (int)(i % M);
    const int c = (int)((i / M) % M);
    const int dir = (int)((i / ((long)M * M)) % 9);
    const long j = i / (9L * M * M);
    const int j1 = (int)(j % L1), j2 = (int)(j / L1);
    const int d1 = dir % 3 - 1, d2 = dir / 3 - 1;
    const long J = (long)wrapc(j2 + d2, L2) * L1 + wrapc(j1 + d1, L1);
    gl(A)[(j * M + r) * N + J * M + c] = gl(Y)[i];
  }
}

// ---- probing --------------------------------------------------------------------
// Probe q = col M + k (col = (J1 mod p1) + p1 (J2 mod p2)) is 1 in
// component k of every coarse site of colour col; probes q0 .. q0 + nq - 1
// go to right-hand sides 0 .. nq - 1.
__global__ __launch_bounds__(256) void probe_kernel(double2* __restrict__ e, int c1, int c2, int M, int p1, int p2,
                                                    int q0, int nq) {
  const long Vc = (long)c1 * c2, n = Vc * M;
  GRID_STRIDE(i, n * nq) {
    const int rhs = (int)(i / n);
    const long t = i % n;
    const long J = t / M;
    const int k = (int)(t % M);
    const int col = (int)(J % c1) % p1 + p1 * ((int)(J / c1) % p2);
    const int q = q0 + rhs;
    gl(e)[i] = make_double2((q == col * M + k) ? 1.0 : 0.0, 0.0);
  }
}

// Galerkin product from probe responses z[rhs][j][r] = (P^dag A P e_q)(j, r):
// the block (j, dir) column k is the response to the probe of the colour of
// site j + dir (period p >= 3: the nine sites of a box have distinct colours).
__global__ __launch_bounds__(256) void galerkin_scatter_kernel(double2* __restrict__ Y, const double2* __restrict__ z,
                                                               int c1, int c2, int M, int p1, int p2, int q0, int nq) {
  const long Vc = (long)c1 * c2;
  GRID_STRIDE(i, Vc * 9 * M * M) {
    const int r = (int)(i % M);
    const int k = (int)((i / M) % M);
    const int dir = (int)((i / ((long)M * M)) % 9);
    const long j = i / (9L * M * M);
    const int j1 = (int)(j % c1), j2 = (int)(j / c1);
    const int n1 = wrapc(j1 + dir % 3 - 1, c1), n2 = wrapc(j2 + dir / 3 - 1, c2);
    const int q = (n1 % p1 + p1 * (n2 % p2)) * M + k;
    if (q < q0 || q >= q0 + nq) continue;
    gl(Y)[i] = gl(z)[(long)(q - q0) * Vc * M + j * M + r];
  }
}

// Smoothed P from responses y[rhs] = (1 - omega A) P_tent e_q (fine layout
// lf): slot (a1, a2) of row (s, d) column k is the response of the probe of
// its block's colour (period >= 2: the widened blocks of one colour are
// disjoint); slots whose block does not reach s are zero.
__global__ __launch_bounds__(256) void psa_scatter_kernel(double2* __restrict__ P, const double2* __restrict__ y,
                                                          NGeom g, int p1, int p2, int q0, int nq) {
  const long Vf = (long)g.f1 * g.f2;
  const int M = g.M;
  GRID_STRIDE(i, Vf * g.dof * 4 * M) {
    const int k = (int)(i % M);
    const int q = (int)((i / M) % 4);
    const long sd = i / (4L * M);
    const long s = sd / g.dof;
    const int d = (int)(sd % g.dof);
    const int x1 = (int)(s % g.f1), x2 = (int)(s / g.f1);
    bool v1, v2;
    const int J1 = slot_coord(x1, g.b1, g.c1, 1, q & 1, v1);
    const int J2 = slot_coord(x2, g.b2, g.c2, 1, q >> 1, v2);
    if (!(v1 && v2)) {
      if (q0 == 0) gl(P)[i] = make_double2(0.0, 0.0);
      continue;
    }
    const int pq = (J1 % p1 + p1 * (J2 % p2)) * M + k;
    if (pq < q0 || pq >= q0 + nq) continue;
    gl(P)[i] = gl(y)[(long)(pq - q0) * Vf * g.dof + g.lf.off(s, d)];
  }
}

// dense[(s dof + d) (Vc M) + J M + k] = P (zeroed before)
__global__ __launch_bounds__(256) void p_dense_kernel(double2* __restrict__ out, const double2* __restrict__ P,
                                                      NGeom g) {
  const int NS = g.sa ? 4 : 1, M = g.M;
  const long Vf = (long)g.f1 * g.f2, cols = (long)g.c1 * g.c2 * M;
  GRID_STRIDE(i, Vf * g.dof * NS * M) {
    const int k = (int)(i % M);
    const int q = (int)((i / M) % NS);
    const long sd = i / ((long)NS * M);
    const long s = sd / g.dof;
    bool v1, v2;
    const int J1 = slot_coord((int)(s % g.f1), g.b1, g.c1, g.sa, q & 1, v1);
    const int J2 = slot_coord((int)(s / g.f1), g.b2, g.c2, g.sa, q >> 1, v2);
    if (!(v1 && v2)) continue;
    gl(out)[sd * cols + ((long)J2 * g.c1 + J1) * M + k] = gl(P)[i];
  }
}

// ---- vector kernels ----------------------------------------------------------------
// scal[slot] = Re <a, b>, scal[slot + 1] = Im <a, b>, scal[slot + 2] = <a, a>
__global__ __launch_bounds__(256) void dot3_kernel(const double2* __restrict__ a, const double2* __restrict__ b, long n,
                                                   RedArgs red, const int* stop) {
  if (stop && *gl(stop)) return;
  double acc[3] = {0.0, 0.0, 0.0};
  gptr<const double2> pa = gl(a), pb = gl(b);
  GRID_STRIDE(i, n) {
    const double2 u = pa[i], v = pb[i];
    acc[0] += u.x * v.x + u.y * v.y;
    acc[1] += u.x * v.y - u.y * v.x;
    acc[2] += u.x * u.x + u.y * u.y;
  }
  double tot[3];
  if (grid_reduce<3>(acc, red.part, red.ticket, 0, tot) && threadIdx.x == 0) {
    gptr<double> sc = gl(red.scal);
    sc[red.slot] = tot[0];
    sc[red.slot + 1] = tot[1];
    sc[red.slot + 2] = tot[2];
  }
}

// CG direction and update guarded by a device stop flag (see kernels.h)
__global__ __launch_bounds__(256) void cgb_dir_kernel(double2* __restrict__ p, const double2* __restrict__ z, long n,
                                                      const double* __restrict__ scal, int gnew, int gold, int fresh,
                                                      const int* stop) {
  if (*gl(stop)) return;
  const double go = scal[gold];
  const double beta = (fresh || !(go > 0.0)) ? 0.0 : scal[gnew] / go;
  GRID_STRIDE(i, n) {
    const double2 zi = z[i];
    double2 pi = fresh ? make_double2(0.0, 0.0) : p[i];
    p[i] = make_double2(zi.x + beta * pi.x, zi.y + beta * pi.y);
  }
}

__global__ __launch_bounds__(256) void cgb_update_kernel(double2* __restrict__ x, double2* __restrict__ r,
                                                         const double2* __restrict__ p, const double2* __restrict__ q,
                                                         long n, RedArgs red, int gamma, int qq, int rr, int rr2,
                                                         double tol2, int* stop, int* iters) {
  if (*gl(stop)) return;
  gptr<double> sc = gl(red.scal);
  const double pq = sc[qq];
  const double a = pq > 0.0 ? sc[gamma] / pq : 0.0;
  double acc[1] = {0.0};
  GRID_STRIDE(i, n) {
    const double2 pi = p[i], qi = q[i];
    double2 xi = x[i], ri = r[i];
    xi.x += a * pi.x;
    xi.y += a * pi.y;
    ri.x -= a * qi.x;
    ri.y -= a * qi.y;
    x[i] = xi;
    r[i] = ri;
    acc[0] += ri.x * ri.x + ri.y * ri.y;
  }
  double tot[1];
  if (grid_reduce<1>(acc, red.part, red.ticket, 0, tot) && threadIdx.x == 0) {
    sc[rr] = tot[0];
    if (rr2 >= 0) sc[rr2] = tot[0];
    gl(iters)[0] += 1;
    if (tot[0] <= tol2) gl(stop)[0] = 1;
  }
}

// minimal-residual step with alpha = omega <p, r> / <p, p> from dot3(p, r):
// x += alpha r, r -= alpha p
__global__ __launch_bounds__(256) void mr_kernel(double2* __restrict__ x, double2* __restrict__ r,
                                                 const double2* __restrict__ p, const double* __restrict__ scal,
                                                 int slot, double omega, long n) {
  const double pp = scal[slot + 2];
  const double s = pp > 0.0 ? omega / pp : 0.0;
  const double ar = s * scal[slot], ai = s * scal[slot + 1];
  GRID_STRIDE(i, n) {
    const double2 ri = r[i], pi = p[i];
    double2 xi = x[i];
    xi.x += ar * ri.x - ai * ri.y;
    xi.y += ar * ri.y + ai * ri.x;
    x[i] = xi;
    r[i] = make_double2(ri.x - (ar * pi.x - ai * pi.y), ri.y - (ar * pi.y + ai * pi.x));
  }
}

// smoother steps: first x = tau b, r = b - tau t; then x += tau r, r -= tau t
__global__ __launch_bounds__(256) void smooth_step_kernel(double2* __restrict__ x, double2* __restrict__ r,
                                                          const double2* __restrict__ b, const double2* __restrict__ t,
                                                          double tau, long n, int first, const int* stop) {
  if (stop && *gl(stop)) return;
  GRID_STRIDE(i, n) {
    const double2 ti = t[i];
    const double2 ri = first ? b[i] : r[i];
    double2 xi = first ? make_double2(0.0, 0.0) : x[i];
    xi.x += tau * ri.x;
    xi.y += tau * ri.y;
    x[i] = xi;
    r[i] = make_double2(ri.x - tau * ti.x, ri.y - tau * ti.y);
  }
}

// x += c1 r - c2 t
__global__ __launch_bounds__(256) void smooth_post_kernel(double2* __restrict__ x, const double2* __restrict__ r,
                                                          const double2* __restrict__ t, double c1, double c2,
                                                          long n, const int* stop) {
  if (stop && *gl(stop)) return;
  GRID_STRIDE(i, n) {
    const double2 ri = r[i], ti = t[i];
    double2 xi = x[i];
    xi.x += c1 * ri.x - c2 * ti.x;
    xi.y += c1 * ri.y - c2 * ti.y;
    x[i] = xi;
  }
}

// y = x + w t (w real)
__global__ __launch_bounds__(256) void axpy3_kernel(double2* __restrict__ y, const double2* __restrict__ x,
                                                    const double2* __restrict__ t, double w, long n) {
  GRID_STRIDE(i, n) {
    const double2 xi = x[i], ti = t[i];
    y[i] = make_double2(xi.x + w * ti.x, xi.y + w * ti.y);
  }
}

// p = q / sqrt(scal[slot + 2])  (the <a, a> of a dot3 of q)
__global__ __launch_bounds__(256) void scale_norm_kernel(double2* __restrict__ p, const double2* __restrict__ q,
                                                         const double* __restrict__ scal, int slot, long n) {
  const double nn = scal[slot + 2];
  const double s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  GRID_STRIDE(i, n) {
    const double2 v = q[i];
    p[i] = make_double2(v.x * s, v.y * s);
  }
}

}  // namespace

size_t normal_orth_lds(const NGeom& g) { return (size_t)g.b1 * g.b2 * g.dof * g.M * sizeof(double2); }

void launch_normal_orth(double2* Pt, const double2* vecs, const NGeom& g, long vstride, int* err, hipStream_t st) {
  const long Vc = (long)g.c1 * g.c2;
  hipLaunchKernelGGL(orth_kernel, dim3((unsigned)Vc), dim3(64), normal_orth_lds(g), st, Pt, vecs, g, vstride, err);
}

void launch_normal_prolong(double2* out, const double2* in, const double2* P, const NGeom& g, int nrhs, int accumulate,
                           hipStream_t st, const int* stop) {
  hipLaunchKernelGGL(prolong_kernel, dim3(nblk((long)g.f1 * g.f2 * g.dof), (unsigned)nrhs), dim3(256), 0, st, out, in,
                     P, g, accumulate, stop);
}

void launch_normal_restrict(double2* out, const double2* in, const double2* P, const NGeom& g, int nrhs,
                            hipStream_t st, const int* stop) {
  const long Vc = (long)g.c1 * g.c2;
  hipLaunchKernelGGL(restrict_kernel, dim3((unsigned)((Vc + 3) / 4), (unsigned)nrhs), dim3(256), 0, st, out, in, P,
                     g, stop);
}

void launch_box(const BoxArgs& a, int nrhs, hipStream_t st) {
  const long V = (long)a.L1 * a.L2;
  if (a.M >= 3 && a.M <= 8)
    hipLaunchKernelGGL(box_wave_kernel, dim3((unsigned)((V + 3) / 4), (unsigned)nrhs), dim3(256), 0, st, a);
  else if (a.M == 2)
    hipLaunchKernelGGL(box2_kernel, dim3(nblk(V), (unsigned)nrhs), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(box_kernel, dim3(nblk(V * a.M), (unsigned)nrhs), dim3(256), 0, st, a);
}

void launch_box_dense(double2* A, const double2* Y, int L1, int L2, int M, hipStream_t st) {
  hipLaunchKernelGGL(box_dense_kernel, dim3(nblk((long)L1 * L2 * 9 * M * M)), dim3(256), 0, st, A, Y, L1, L2, M);
}

void launch_probe(double2* e, int c1, int c2, int M, int p1, int p2, int q0, int nq, hipStream_t st) {
  hipLaunchKernelGGL(probe_kernel, dim3(nblk((long)c1 * c2 * M * nq)), dim3(256), 0, st, e, c1, c2, M, p1, p2, q0,
                     nq);
}

void launch_galerkin_box_scatter(double2* Y, const double2* z, int c1, int c2, int M, int p1, int p2, int q0, int nq,
                                 hipStream_t st) {
  hipLaunchKernelGGL(galerkin_scatter_kernel, dim3(nblk((long)c1 * c2 * 9 * M * M)), dim3(256), 0, st, Y, z, c1, c2,
                     M, p1, p2, q0, nq);
}

void launch_psa_scatter(double2* P, const double2* y, const NGeom& g, int p1, int p2, int q0, int nq,
                        hipStream_t st) {
  hipLaunchKernelGGL(psa_scatter_kernel, dim3(nblk((long)g.f1 * g.f2 * g.dof * 4 * g.M)), dim3(256), 0, st, P, y, g,
                     p1, p2, q0, nq);
}

void launch_normal_p_dense(double2* out, const double2* P, const NGeom& g, hipStream_t st) {
  const long n = (long)g.f1 * g.f2 * g.dof * (g.sa ? 4 : 1) * g.M;
  hipLaunchKernelGGL(p_dense_kernel, dim3(nblk(n)), dim3(256), 0, st, out, P, g);
}

void launch_dot3(const double2* a, const double2* b, long n, RedArgs red, hipStream_t st, const int* stop) {
  long nb = (n + 255) / 256;
  const long cap = red_block_cap();
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(dot3_kernel, dim3((unsigned)nb), dim3(256), 0, st, a, b, n, red, stop);
}

void launch_cgb_dir(double2* p, const double2* z, long n, const double* scal, int gnew, int gold, int fresh,
                    const int* stop, hipStream_t st) {
  hipLaunchKernelGGL(cgb_dir_kernel, dim3(nblk(n)), dim3(256), 0, st, p, z, n, scal, gnew, gold, fresh, stop);
}

void launch_cgb_update(double2* x, double2* r, const double2* p, const double2* q, long n, RedArgs red, int gamma,
                       int qq, int rr, int rr2, double tol2, int* stop, int* iters, hipStream_t st) {
  long nb = (n + 255) / 256;
  const long cap = red_block_cap();
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(cgb_update_kernel, dim3((unsigned)nb), dim3(256), 0, st, x, r, p, q, n, red, gamma, qq, rr, rr2,
                     tol2, stop, iters);
}

void launch_mr_step(double2* x, double2* r, const double2* p, const double* scal, int slot, double omega, long n,
                    hipStream_t st) {
  hipLaunchKernelGGL(mr_kernel, dim3(nblk(n)), dim3(256), 0, st, x, r, p, scal, slot, omega, n);
}

void launch_smooth_step(double2* x, double2* r, const double2* b, const double2* t, double tau, long n, int first,
                        hipStream_t st, const int* stop) {
  hipLaunchKernelGGL(smooth_step_kernel, dim3(nblk(n)), dim3(256), 0, st, x, r, b, t, tau, n, first, stop);
}

void launch_smooth_post(double2* x, const double2* r, const double2* t, double c1, double c2, long n,
                        hipStream_t st, const int* stop) {
  hipLaunchKernelGGL(smooth_post_kernel, dim3(nblk(n)), dim3(256), 0, st, x, r, t, c1, c2, n, stop);
}

void launch_axpy3(double2* y, const double2* x, const double2* t, double w, long n, hipStream_t st) {
  hipLaunchKernelGGL(axpy3_kernel, dim3(nblk(n)), dim3(256), 0, st, y, x, t, w, n);
}

void launch_scale_norm(double2* p, const double2* q, const double* scal, int slot, long n, hipStream_t st) {
  hipLaunchKernelGGL(scale_norm_kernel, dim3(nblk(n)), dim3(256), 0, st, p, q, scal, slot, n);
}

}  // namespace amg

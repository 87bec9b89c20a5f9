// Four-dimensional SU(3) Wilson-Dirac stencil on gfx950 (chiral gamma basis).
//
//   (D psi)(x) = (4 + m) psi(x)
//     - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// With gamma_mu = [[0, B_mu], [B_mu^dag, 0]] and gamma_mu^2 = 1, the
// projector 1 + s gamma_mu (s = +-1) maps psi to (h, s B_mu^dag h) with the
// half spinor h = psi_up + s B_mu psi_down, so each hop multiplies only two
// colour vectors by the link:
//   mu = 1: h = (p0 - i s p3, p1 - i s p2), lower = (i s u1, i s u0)
//   mu = 2: h = (p0 - s p3,   p1 + s p2),   lower = (s u1, -s u0)
//   mu = 3: h = (p0 - i s p2, p1 + i s p3), lower = (i s u0, -i s u1)
//   mu = 4: h = (p0 + s p2,   p1 + s p3),   lower = (s u0, s u1)
// where u = U h (forward hop) or U^dag h (backward hop).
//
// Internal layouts (component index = spin * 3 + colour):
//   FP64 spinor: 12 planes [comp][site] of double2        (Layout{V, 12, 1})
//   FP32 spinor: 6 planes [comp/2][site] of float4         (Layout{V, 12, 2})
//   links: 36 planes [mu*9 + a*3 + b][site] (double2 / float2)
#include <cstdlib>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace amg {
namespace {

template <typename T> struct Spinor { cplx<T> c[4][3]; };

__device__ __forceinline__ void ld_spinor(gptr<const double2> __restrict__ p, long s, long V, Spinor<double>& o) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.c[sp][c] = p[(long)(sp * 3 + c) * V + s];
}
__device__ __forceinline__ void ld_spinor(gptr<const float2> __restrict__ p, long s, long V, Spinor<float>& o) {
  gptr<const float4> q = (gptr<const float4>)p;
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const float4 v = q[(long)u * V + s];
    const int c0 = 2 * u, c1 = 2 * u + 1;
    o.c[c0 / 3][c0 % 3] = make_float2(v.x, v.y);
    o.c[c1 / 3][c1 % 3] = make_float2(v.z, v.w);
  }
}
__device__ __forceinline__ void st_spinor(gptr<double2> __restrict__ p, long s, long V, const Spinor<double>& o) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[(long)(sp * 3 + c) * V + s] = o.c[sp][c];
}
__device__ __forceinline__ void st_spinor(gptr<float2> __restrict__ p, long s, long V, const Spinor<float>& o) {
  gptr<float4> q = (gptr<float4>)p;
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int c0 = 2 * u, c1 = 2 * u + 1;
    const float2 a = o.c[c0 / 3][c0 % 3], b = o.c[c1 / 3][c1 % 3];
    q[(long)u * V + s] = make_float4(a.x, a.y, b.x, b.y);
  }
}

// streaming (non-temporal) stores for lattices far larger than the caches:
// the result bypasses L2, so it evicts no neighbour data and leaves no dirty
// lines for the reductions' release fences to write back
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st_spinor_nt(gptr<double2> __restrict__ p, long s, long V, const Spinor<double>& o) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const v2d v = {o.c[sp][c].x, o.c[sp][c].y};
      __builtin_nontemporal_store(v, (gptr<v2d>)p + (long)(sp * 3 + c) * V + s);
    }
}
__device__ __forceinline__ void st_spinor_nt(gptr<float2> __restrict__ p, long s, long V, const Spinor<float>& o) {
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int c0 = 2 * u, c1 = 2 * u + 1;
    const float2 a = o.c[c0 / 3][c0 % 3], b = o.c[c1 / 3][c1 % 3];
    const v4f v = {a.x, a.y, b.x, b.y};
    __builtin_nontemporal_store(v, (gptr<v4f>)p + (long)u * V + s);
  }
}
template <bool NT, typename T>
__device__ __forceinline__ void st_out(gptr<cplx<T>> __restrict__ p, long s, long V, const Spinor<T>& o) {
  if (NT) st_spinor_nt(p, s, V, o);
  else st_spinor(p, s, V, o);
}

// <o, c>, |o|^2 (MRDOT) or |o|^2 (NORM) of one site, summed over its 12
// components in T and added to the FP64 accumulators
template <typename T, int EPI>
__device__ __forceinline__ void site_dots(const Spinor<T>& o, const Spinor<T>& c, double (&acc)[3]) {
  T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cplx<T> u = o.c[sp][k], r = c.c[sp][k];
      if (EPI == EPI_MRDOT) {
        s0 += u.x * r.x + u.y * r.y;
        s1 += u.x * r.y - u.y * r.x;
      }
      s2 += u.x * u.x + u.y * u.y;
    }
  if (EPI == EPI_MRDOT) {
    acc[0] += (double)s0;
    acc[1] += (double)s1;
    acc[2] += (double)s2;
  } else {
    acc[0] += (double)s2;
  }
}

template <typename T> struct Link { cplx<T> m[3][3]; };

template <typename T>
__device__ __forceinline__ void ld_link(gptr<const cplx<T>> __restrict__ U, long s, long V, int mu, Link<T>& L) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) L.m[a][b] = U[(long)(mu * 9 + a * 3 + b) * V + s];
}

// third row of an SU(3) matrix from the first two: r2 = conj(r0 x r1)
template <typename T>
__device__ __forceinline__ void su3_third_row(Link<T>& L) {
  const cplx<T> a = csub<T>(cmul<T>(L.m[0][1], L.m[1][2]), cmul<T>(L.m[0][2], L.m[1][1]));
  const cplx<T> b = csub<T>(cmul<T>(L.m[0][2], L.m[1][0]), cmul<T>(L.m[0][0], L.m[1][2]));
  const cplx<T> c = csub<T>(cmul<T>(L.m[0][0], L.m[1][1]), cmul<T>(L.m[0][1], L.m[1][0]));
  L.m[2][0] = mk<T>(a.x, -a.y);
  L.m[2][1] = mk<T>(b.x, -b.y);
  L.m[2][2] = mk<T>(c.x, -c.y);
}
// two-row links: three 16-byte loads (FP32) or six (FP64) per link
__device__ __forceinline__ void ld_link_c(const void* Uc, long s, long V, int mu, Link<float>& L) {
  gptr<const float4> q = (gptr<const float4>)Uc + (long)(mu * 3) * V + s;
  const float4 q0 = q[0], q1 = q[V], q2 = q[2 * V];
  L.m[0][0] = make_float2(q0.x, q0.y); L.m[0][1] = make_float2(q0.z, q0.w);
  L.m[0][2] = make_float2(q1.x, q1.y); L.m[1][0] = make_float2(q1.z, q1.w);
  L.m[1][1] = make_float2(q2.x, q2.y); L.m[1][2] = make_float2(q2.z, q2.w);
  su3_third_row<float>(L);
}
__device__ __forceinline__ void ld_link_c(const void* Uc, long s, long V, int mu, Link<double>& L) {
  gptr<const double2> q = (gptr<const double2>)Uc + (long)(mu * 6) * V + s;
#pragma unroll
  for (int e = 0; e < 6; ++e) L.m[e / 3][e % 3] = q[(long)e * V];
  su3_third_row<double>(L);
}
template <typename T, bool COMP>
__device__ __forceinline__ void ld_lnk(gptr<const cplx<T>> __restrict__ U, const void* Uc, long s, long V, int mu,
                                       Link<T>& L) {
  if (COMP) ld_link_c(Uc, s, V, mu, L);
  else ld_link<T>(U, s, V, mu, L);
}

// o += -1/2 * (1 + s gamma_mu) W psi, W = U (DAGU = false) or U^dag (true)
template <typename T, int MU, bool DAGU>
__device__ __forceinline__ void hop(Spinor<T>& o, const Spinor<T>& p, const Link<T>& L, T s) {
  cplx<T> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<T> p0 = p.c[0][c], p1 = p.c[1][c], p2 = p.c[2][c], p3 = p.c[3][c];
    if (MU == 0) {        // h0 = p0 - i s p3, h1 = p1 - i s p2
      h0[c] = mk<T>(p0.x + s * p3.y, p0.y - s * p3.x);
      h1[c] = mk<T>(p1.x + s * p2.y, p1.y - s * p2.x);
    } else if (MU == 1) { // h0 = p0 - s p3, h1 = p1 + s p2
      h0[c] = mk<T>(p0.x - s * p3.x, p0.y - s * p3.y);
      h1[c] = mk<T>(p1.x + s * p2.x, p1.y + s * p2.y);
    } else if (MU == 2) { // h0 = p0 - i s p2, h1 = p1 + i s p3
      h0[c] = mk<T>(p0.x + s * p2.y, p0.y - s * p2.x);
      h1[c] = mk<T>(p1.x - s * p3.y, p1.y + s * p3.x);
    } else {              // h0 = p0 + s p2, h1 = p1 + s p3
      h0[c] = mk<T>(p0.x + s * p2.x, p0.y + s * p2.y);
      h1[c] = mk<T>(p1.x + s * p3.x, p1.y + s * p3.y);
    }
  }
  cplx<T> u0[3], u1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<T> x0 = mk<T>(0, 0), x1 = mk<T>(0, 0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (DAGU) {
        cjfma<T>(x0, L.m[b][a], h0[b]);
        cjfma<T>(x1, L.m[b][a], h1[b]);
      } else {
        cfma<T>(x0, L.m[a][b], h0[b]);
        cfma<T>(x1, L.m[a][b], h1[b]);
      }
    }
    u0[a] = x0; u1[a] = x1;
  }
  const T hf = (T)0.5;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cplx<T> l2, l3;
    if (MU == 0) { l2 = cscale<T>(s, ctimesi<T>(u1[c])); l3 = cscale<T>(s, ctimesi<T>(u0[c])); }
    else if (MU == 1) { l2 = cscale<T>(s, u1[c]); l3 = cscale<T>(-s, u0[c]); }
    else if (MU == 2) { l2 = cscale<T>(s, ctimesi<T>(u0[c])); l3 = cscale<T>(-s, ctimesi<T>(u1[c])); }
    else { l2 = cscale<T>(s, u0[c]); l3 = cscale<T>(s, u1[c]); }
    o.c[0][c].x -= hf * u0[c].x; o.c[0][c].y -= hf * u0[c].y;
    o.c[1][c].x -= hf * u1[c].x; o.c[1][c].y -= hf * u1[c].y;
    o.c[2][c].x -= hf * l2.x;    o.c[2][c].y -= hf * l2.y;
    o.c[3][c].x -= hf * l3.x;    o.c[3][c].y -= hf * l3.y;
  }
}

struct Geo4 {
  int L[4];
  long st[4];
  __device__ __forceinline__ void nb(long s, long* fw, long* bw) const {
    long rem = s;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int x = (int)(rem % L[mu]);
      rem /= L[mu];
      fw[mu] = (x == L[mu] - 1) ? s - (long)(L[mu] - 1) * st[mu] : s + st[mu];
      bw[mu] = (x == 0) ? s + (long)(L[mu] - 1) * st[mu] : s - st[mu];
    }
  }
  __device__ __forceinline__ void coords(long s, int* x) const {
    long rem = s;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) { x[mu] = (int)(rem % L[mu]); rem /= L[mu]; }
  }
};

template <typename T, int DAG, bool COMP>
__device__ __forceinline__ void all_hops(Spinor<T>& o, gptr<const cplx<T>> __restrict__ pin, gptr<const cplx<T>> __restrict__ U,
                                         const void* Uc, long s, long V, const long* fw, const long* bw) {
  const T sf = DAG ? (T)1 : (T)-1, sb = -sf;
  Spinor<T> p;
  Link<T> L;
#define AMG_HOP4(MU)                                  \
  ld_spinor(pin, fw[MU], V, p); ld_lnk<T, COMP>(U, Uc, s, V, MU, L);      hop<T, MU, false>(o, p, L, sf); \
  ld_spinor(pin, bw[MU], V, p); ld_lnk<T, COMP>(U, Uc, bw[MU], V, MU, L); hop<T, MU, true>(o, p, L, sb);
  AMG_HOP4(0) AMG_HOP4(1) AMG_HOP4(2) AMG_HOP4(3)
#undef AMG_HOP4
}

Geo4 geo(const int* d);

// W: minimum waves per SIMD asked of the register allocator
template <typename T, int DAG, int EPI, int W, bool NT, bool COMP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W, 8))) void wilson4d_kernel(
    WilsonArgs<T> a0, const WilsonArgs<T>* batch) {
  AMG_ARGS(WilsonArgs<T>)
  const int rhs = blockIdx.y;
  const RedArgs& red = a.red;
  if (skip_rhs(red.flags, rhs)) return;
  const int d4[4] = {a.L1, a.L2, a.L3, a.L4};
  Geo4 G;
  {
    long st = 1;
    for (int mu = 0; mu < 4; ++mu) { G.L[mu] = d4[mu]; G.st[mu] = st; st *= d4[mu]; }
  }
  const long V = (long)a.L1 * a.L2 * a.L3 * a.L4;
  const long ro = (long)rhs * 12 * V;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ U = gl(a.U);
  gptr<const cplx<T>> __restrict__ bvec = gl(a.b);
  gptr<cplx<T>> __restrict__ out = gl(a.out);
  gptr<cplx<T>> __restrict__ copy_out = gl(a.copy_out);
  const T diag = (T)(4.0 + a.mass);
  double acc[3] = {0.0, 0.0, 0.0};
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (long)gridDim.x * blockDim.x) {
    long fw[4], bw[4];
    G.nb(s, fw, bw);
    Spinor<T> c, o;
    ld_spinor(pin, s, V, c);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) o.c[sp][k] = cscale<T>(diag, c.c[sp][k]);
    all_hops<T, DAG, COMP>(o, pin, U, a.Uc, s, V, fw, bw);
    if (EPI == EPI_RESID) {
      Spinor<T> b;
      ld_spinor(bvec + ro, s, V, b);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) o.c[sp][k] = csub<T>(b.c[sp][k], o.c[sp][k]);
    }
    st_out<NT>(out + ro, s, V, o);
    if (copy_out) st_out<NT>(copy_out + ro, s, V, c);
    if (EPI == EPI_MRDOT || EPI == EPI_NORM) site_dots<T, EPI>(o, c, acc);
  }
  if (EPI == EPI_MRDOT) {
    double tot[3];
    if (grid_reduce<3>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) finalize_mr(tot, red, rhs);
  } else if (EPI == EPI_NORM) {
    double a1[1] = {acc[0]}, tot[1];
    if (grid_reduce<1>(a1, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) red.scal[red.slot + rhs] = tot[0];
  }
}

// The same operator with every thread marching along x_4 over TT sites of one
// (x_1, x_2, x_3) column: the spinors at x_4 - 1 and x_4 and the backward
// x_4 link come from the previous step's registers, so per site only the
// x_4 + 1 spinor is new along x_4 (the t-neighbours of a site lie a whole
// 3-volume apart and would otherwise be re-fetched from memory), and the
// blocks are renumbered so that every XCD works on one contiguous part of
// the lattice (its L2 then holds the x_3 neighbours of its own columns).
// Registers: 233 VGPRs with two-row links (two waves per SIMD); asking the
// allocator for three or four waves spills and measured 1.4-2.3x slower.
template <typename T, int DAG, int EPI, int TT, bool NT, bool COMP>
__global__ __launch_bounds__(256) void wilson4d_tm_kernel(
    WilsonArgs<T> a0, const WilsonArgs<T>* batch) {
  AMG_ARGS(WilsonArgs<T>)
  const int rhs = blockIdx.y;
  const RedArgs& red = a.red;
  if (skip_rhs(red.flags, rhs)) return;
  const int L1 = a.L1, L2 = a.L2, L3 = a.L3, L4 = a.L4;
  const long V3 = (long)L1 * L2 * L3;
  const long V = V3 * L4;
  const long ro = (long)rhs * 12 * V;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ U = gl(a.U);
  const T diag = (T)(4.0 + a.mass);
  const T sf = DAG ? (T)1 : (T)-1, sb = -sf;
  const int nslab = (L4 + TT - 1) / TT;
  const long work = V3 * nslab;
  const long nb = gridDim.x;
  const long lb = (nb % 8 == 0) ? (long)(blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : (long)blockIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  for (long w = lb * blockDim.x + threadIdx.x; w < work; w += nb * blockDim.x) {
    const int slab = (int)(w / V3);
    const long q = w - (long)slab * V3;
    const int x1 = (int)(q % L1), x2 = (int)((q / L1) % L2), x3 = (int)(q / ((long)L1 * L2));
    long qf[3], qb[3];
    qf[0] = (x1 == L1 - 1) ? q - (L1 - 1) : q + 1;
    qb[0] = (x1 == 0) ? q + (L1 - 1) : q - 1;
    qf[1] = (x2 == L2 - 1) ? q - (long)(L2 - 1) * L1 : q + L1;
    qb[1] = (x2 == 0) ? q + (long)(L2 - 1) * L1 : q - L1;
    qf[2] = (x3 == L3 - 1) ? q - (long)(L3 - 1) * L1 * L2 : q + (long)L1 * L2;
    qb[2] = (x3 == 0) ? q + (long)(L3 - 1) * L1 * L2 : q - (long)L1 * L2;
    const int t0 = slab * TT;
    const int t1 = (t0 + TT < L4) ? t0 + TT : L4;
    Spinor<T> prev, cur, nxt, p;
    Link<T> Lb, Lf;
    {
      const long s0 = q + (long)t0 * V3;
      const long sm = q + (long)((t0 + L4 - 1) % L4) * V3;
      ld_spinor(pin, s0, V, cur);
      ld_spinor(pin, sm, V, prev);
      ld_lnk<T, COMP>(U, a.Uc, sm, V, 3, Lb);
    }
    for (int t = t0; t < t1; ++t) {
      const long toff = (long)t * V3;
      const long s = q + toff;
      ld_spinor(pin, q + (long)((t + 1) % L4) * V3, V, nxt);
      ld_lnk<T, COMP>(U, a.Uc, s, V, 3, Lf);
      Spinor<T> o;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) o.c[sp][k] = cscale<T>(diag, cur.c[sp][k]);
      Link<T> L;
#define AMG_HOP3(MU)                                                                                      \
  ld_spinor(pin, qf[MU] + toff, V, p); ld_lnk<T, COMP>(U, a.Uc, s, V, MU, L); hop<T, MU, false>(o, p, L, sf); \
  ld_spinor(pin, qb[MU] + toff, V, p); ld_lnk<T, COMP>(U, a.Uc, qb[MU] + toff, V, MU, L);                   \
  hop<T, MU, true>(o, p, L, sb);
      AMG_HOP3(0) AMG_HOP3(1) AMG_HOP3(2)
#undef AMG_HOP3
      hop<T, 3, false>(o, nxt, Lf, sf);
      hop<T, 3, true>(o, prev, Lb, sb);
      if (EPI == EPI_RESID) {
        Spinor<T> b;
        ld_spinor(gl(a.b) + ro, s, V, b);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) o.c[sp][k] = csub<T>(b.c[sp][k], o.c[sp][k]);
      }
      st_out<NT>(gl(a.out) + ro, s, V, o);
      if (a.copy_out) st_out<NT>(gl(a.copy_out) + ro, s, V, cur);
      if (EPI == EPI_MRDOT || EPI == EPI_NORM) site_dots<T, EPI>(o, cur, acc);
      prev = cur;
      cur = nxt;
      Lb = Lf;
    }
  }
  if (EPI == EPI_MRDOT) {
    double tot[3];
    if (grid_reduce<3>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) finalize_mr(tot, red, rhs);
  } else if (EPI == EPI_NORM) {
    double a1[1] = {acc[0]}, tot[1];
    if (grid_reduce<1>(a1, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) red.scal[red.slot + rhs] = tot[0];
  }
}

// Split apply for the Galerkin product (FP64): out[0] = diagonal + hops inside
// the block, out[1 + dir] = hop in direction dir leaving the block.
__global__ __launch_bounds__(256) void wilson4d_split_kernel(double2* __restrict__ out_, const double2* __restrict__ in,
                                                             const double2* __restrict__ U_, double diag, Geo4 G, long V,
                                                             int b0, int b1, int b2, int b3, int nrhs) {
  const int rhs = blockIdx.y;
  const long ro = (long)rhs * 12 * V;
  const long ks = (long)nrhs * 12 * V;
  const int blk[4] = {b0, b1, b2, b3};
  gptr<const double2> __restrict__ pin = gl(in) + ro;
  gptr<const double2> __restrict__ U = gl(U_);
  gptr<double2> __restrict__ out = gl(out_);
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (long)gridDim.x * blockDim.x) {
    long fw[4], bw[4];
    int x[4];
    G.nb(s, fw, bw);
    G.coords(s, x);
    Spinor<double> c, o, t, p;
    Link<double> L;
    ld_spinor(pin, s, V, c);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) o.c[sp][k] = cscale<double>(diag, c.c[sp][k]);
    auto route = [&](int dir, bool cross) {
      if (cross) {
        st_spinor(out + (long)(1 + dir) * ks + ro, s, V, t);
      } else {
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) o.c[sp][k] = cadd<double>(o.c[sp][k], t.c[sp][k]);
        Spinor<double> z;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int k = 0; k < 3; ++k) z.c[sp][k] = mk<double>(0, 0);
        st_spinor(out + (long)(1 + dir) * ks + ro, s, V, z);
      }
    };
    auto zero_t = [&]() {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) t.c[sp][k] = mk<double>(0, 0);
    };
#define AMG_SPLIT4(MU)                                                                              \
  zero_t(); ld_spinor(pin, fw[MU], V, p); ld_link<double>(U, s, V, MU, L);                          \
  hop<double, MU, false>(t, p, L, -1.0); route(2 * MU, x[MU] % blk[MU] == blk[MU] - 1);             \
  zero_t(); ld_spinor(pin, bw[MU], V, p); ld_link<double>(U, bw[MU], V, MU, L);                     \
  hop<double, MU, true>(t, p, L, 1.0); route(2 * MU + 1, x[MU] % blk[MU] == 0);
    AMG_SPLIT4(0) AMG_SPLIT4(1) AMG_SPLIT4(2) AMG_SPLIT4(3)
#undef AMG_SPLIT4
    st_spinor(out + ro, s, V, o);
  }
}

__global__ void links4d_pack_kernel(double2* __restrict__ U64, float2* __restrict__ U32, const double2* __restrict__ c,
                                    long V) {
  const long total = 4 * V;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
#pragma unroll
    for (int ab = 0; ab < 9; ++ab) {
      const double2 z = c[i * 9 + ab];
      U64[(long)(mu * 9 + ab) * V + s] = z;
      U32[(long)(mu * 9 + ab) * V + s] = make_float2((float)z.x, (float)z.y);
    }
  }
}

// Two-row copies of the links and the SU(3) check (FP64: |U U^dag - 1| and
// |det U - 1| below 1e-9 for every link, else the flag is raised and the
// caller keeps the full links).
__global__ void links4d_compress_kernel(double2* __restrict__ Uc64, float4* __restrict__ Uc32,
                                        const double2* __restrict__ c, long V, int* __restrict__ not_su3) {
  const long total = 4 * V;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int mu = (int)(i / V);
    const long s = i - (long)mu * V;
    double2 m[3][3];
#pragma unroll
    for (int ab = 0; ab < 9; ++ab) m[ab / 3][ab % 3] = c[i * 9 + ab];
    double dev = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double2 acc = make_double2(a == b ? -1.0 : 0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {   // (U U^dag)_ab = sum_k U_ak conj(U_bk)
          acc.x += m[a][k].x * m[b][k].x + m[a][k].y * m[b][k].y;
          acc.y += m[a][k].y * m[b][k].x - m[a][k].x * m[b][k].y;
        }
        dev = fmax(dev, fabs(acc.x) + fabs(acc.y));
      }
    const double2 c0 = csub<double>(cmul<double>(m[1][1], m[2][2]), cmul<double>(m[1][2], m[2][1]));
    const double2 c1 = csub<double>(cmul<double>(m[1][2], m[2][0]), cmul<double>(m[1][0], m[2][2]));
    const double2 c2 = csub<double>(cmul<double>(m[1][0], m[2][1]), cmul<double>(m[1][1], m[2][0]));
    double2 det = cmul<double>(m[0][0], c0);
    det = cadd<double>(det, cmul<double>(m[0][1], c1));
    det = cadd<double>(det, cmul<double>(m[0][2], c2));
    dev = fmax(dev, fabs(det.x - 1.0) + fabs(det.y));
    if (!(dev <= 1e-9)) atomicOr(not_su3, 1);
#pragma unroll
    for (int e = 0; e < 6; ++e) Uc64[(long)(mu * 6 + e) * V + s] = m[e / 3][e % 3];
    Uc32[(long)(mu * 3 + 0) * V + s] = make_float4((float)m[0][0].x, (float)m[0][0].y, (float)m[0][1].x, (float)m[0][1].y);
    Uc32[(long)(mu * 3 + 1) * V + s] = make_float4((float)m[0][2].x, (float)m[0][2].y, (float)m[1][0].x, (float)m[1][0].y);
    Uc32[(long)(mu * 3 + 2) * V + s] = make_float4((float)m[1][1].x, (float)m[1][1].y, (float)m[1][2].x, (float)m[1][2].y);
  }
}

Geo4 geo(const int* d) {
  Geo4 G;
  long st = 1;
  for (int mu = 0; mu < 4; ++mu) { G.L[mu] = d[mu]; G.st[mu] = st; st *= d[mu]; }
  return G;
}

}  // namespace

// t-march length: 16 for FP32 (measured ~5% faster than one site per
// thread at 32^3 x 64); 0 (one site per thread) for FP64, where the three
// register-resident spinors spill
template <typename T>
int w4_tt() {
  static int tt = [] {
    const char* e = std::getenv("AMG_W4_TT");
    return e ? std::atoi(e) : (sizeof(T) == 4 ? 16 : 0);
  }();
  return tt;
}
// minimum waves per SIMD for the one-site kernel: 2 for FP32 (fits without
// spilling, ~10% faster), 1 for FP64 (two waves would spill)
template <typename T>
int w4_waves() {
  static int w = [] {
    const char* e = std::getenv("AMG_W4_WAVES");
    return e ? std::atoi(e) : (sizeof(T) == 4 ? 2 : 1);
  }();
  return w;
}

template <typename T>
void launch_wilson4d(const WilsonArgs<T>& a, int dagger, int epi, hipStream_t st) {
  const long V = (long)a.L1 * a.L2 * a.L3 * a.L4;
  const bool red = (epi == EPI_MRDOT || epi == EPI_NORM);
  // reducing epilogues: FP32 marches 16 sites along x_4 (the 12-rhs MR
  // smoother at 32^3 x 64: solve 9.54 -> 9.09 s against one site per
  // thread), FP64 runs one site per thread (its marching form is slower)
  static const int tt_red = [] {
    const char* e = std::getenv("AMG_W4_TT_RED");
    return e ? std::atoi(e) : (sizeof(T) == 4 ? 16 : 0);
  }();
  const int tt = (red && tt_red >= 0) ? tt_red : w4_tt<T>();
  const bool nt = V >= (1L << 20);
  const bool comp = a.Uc != nullptr;
  if (tt == 4 || tt == 8 || tt == 16) {
    const long V3 = (long)a.L1 * a.L2 * a.L3;
    long nb = (V3 * ((a.L4 + tt - 1) / tt) + 255) / 256;
    if (red) nb = nb < red_block_cap() ? nb : red_block_cap();
    dim3 grid((unsigned)nb, (unsigned)a.nrhs);
// (streaming stores measured 2x slower in the x_4-marching kernel: 548 vs
// 276 us at 32^3 x 64; it keeps ordinary stores)
#define AMG_W4T(TT, DAG, EPI)                                                                  \
  if (comp) { dispatch(wilson4d_tm_kernel<T, DAG, EPI, TT, false, true>, a, grid, dim3(256), st); } \
  else { dispatch(wilson4d_tm_kernel<T, DAG, EPI, TT, false, false>, a, grid, dim3(256), st); }
#define AMG_W4T_E(TT, DAG)                                   \
    switch (epi) {                                          \
      case EPI_PLAIN: AMG_W4T(TT, DAG, EPI_PLAIN); break;   \
      case EPI_MRDOT: AMG_W4T(TT, DAG, EPI_MRDOT); break;   \
      case EPI_RESID: AMG_W4T(TT, DAG, EPI_RESID); break;   \
      default: AMG_W4T(TT, DAG, EPI_NORM); break;           \
    }
#define AMG_W4T_D(TT) if (dagger) { AMG_W4T_E(TT, 1) } else { AMG_W4T_E(TT, 0) }
    if (tt == 4) { AMG_W4T_D(4) } else if (tt == 8) { AMG_W4T_D(8) } else { AMG_W4T_D(16) }
#undef AMG_W4T_D
#undef AMG_W4T_E
#undef AMG_W4T
    return;
  }
  long nb = (V + 255) / 256;
  if (red) nb = nb < red_block_cap() ? nb : red_block_cap();
  dim3 grid((unsigned)nb, (unsigned)a.nrhs);
#define AMG_W4N(DAG, EPI, W)                                                                          \
  if (nt) {                                                                                          \
    if (comp) { dispatch(wilson4d_kernel<T, DAG, EPI, W, true, true>, a, grid, dim3(256), st); }     \
    else { dispatch(wilson4d_kernel<T, DAG, EPI, W, true, false>, a, grid, dim3(256), st); }         \
  } else {                                                                                           \
    if (comp) { dispatch(wilson4d_kernel<T, DAG, EPI, W, false, true>, a, grid, dim3(256), st); }    \
    else { dispatch(wilson4d_kernel<T, DAG, EPI, W, false, false>, a, grid, dim3(256), st); }        \
  }
#define AMG_W4(DAG, EPI) if (w2) { AMG_W4N(DAG, EPI, 2); } else { AMG_W4N(DAG, EPI, 1); }
  const bool w2 = w4_waves<T>() == 2;
  if (dagger) {
    switch (epi) {
      case EPI_PLAIN: AMG_W4(1, EPI_PLAIN); break;
      case EPI_MRDOT: AMG_W4(1, EPI_MRDOT); break;
      case EPI_RESID: AMG_W4(1, EPI_RESID); break;
      default: AMG_W4(1, EPI_NORM); break;
    }
  } else {
    switch (epi) {
      case EPI_PLAIN: AMG_W4(0, EPI_PLAIN); break;
      case EPI_MRDOT: AMG_W4(0, EPI_MRDOT); break;
      case EPI_RESID: AMG_W4(0, EPI_RESID); break;
      default: AMG_W4(0, EPI_NORM); break;
    }
  }
#undef AMG_W4
#undef AMG_W4N
}
template void launch_wilson4d<double>(const WilsonArgs<double>&, int, int, hipStream_t);
template void launch_wilson4d<float>(const WilsonArgs<float>&, int, int, hipStream_t);

void launch_wilson4d_split(double2* out, const double2* in, const double2* U, double mass, const int* dims,
                           const int* blk, int nrhs, hipStream_t st) {
  const Geo4 G = geo(dims);
  const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
  dim3 grid((unsigned)((V + 255) / 256), (unsigned)nrhs);
  hipLaunchKernelGGL(wilson4d_split_kernel, grid, dim3(256), 0, st, out, in, U, 4.0 + mass, G, V, blk[0], blk[1],
                     blk[2], blk[3], nrhs);
}

void launch_links4d_compress(double2* Uc64, float4* Uc32, const double2* canon, long V, int* not_su3,
                             hipStream_t st) {
  long nb = (4 * V + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(links4d_compress_kernel, dim3((unsigned)nb), dim3(256), 0, st, Uc64, Uc32, canon, V, not_su3);
}

void launch_links4d_pack(double2* U64, float2* U32, const double2* canon, long V, hipStream_t st) {
  long nb = (4 * V + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(links4d_pack_kernel, dim3((unsigned)nb), dim3(256), 0, st, U64, U32, canon, V);
}

}  // namespace amg

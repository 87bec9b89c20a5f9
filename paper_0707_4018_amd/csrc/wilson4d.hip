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
#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace amg {
namespace {

template <typename T> struct Spinor { cplx<T> c[4][3]; };

__device__ __forceinline__ void ld_spinor(const double2* __restrict__ p, long s, long V, Spinor<double>& o) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.c[sp][c] = p[(long)(sp * 3 + c) * V + s];
}
__device__ __forceinline__ void ld_spinor(const float2* __restrict__ p, long s, long V, Spinor<float>& o) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const float4 v = q[(long)u * V + s];
    const int c0 = 2 * u, c1 = 2 * u + 1;
    o.c[c0 / 3][c0 % 3] = make_float2(v.x, v.y);
    o.c[c1 / 3][c1 % 3] = make_float2(v.z, v.w);
  }
}
__device__ __forceinline__ void st_spinor(double2* __restrict__ p, long s, long V, const Spinor<double>& o) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[(long)(sp * 3 + c) * V + s] = o.c[sp][c];
}
__device__ __forceinline__ void st_spinor(float2* __restrict__ p, long s, long V, const Spinor<float>& o) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int c0 = 2 * u, c1 = 2 * u + 1;
    const float2 a = o.c[c0 / 3][c0 % 3], b = o.c[c1 / 3][c1 % 3];
    q[(long)u * V + s] = make_float4(a.x, a.y, b.x, b.y);
  }
}

template <typename T> struct Link { cplx<T> m[3][3]; };

template <typename T>
__device__ __forceinline__ void ld_link(const cplx<T>* __restrict__ U, long s, long V, int mu, Link<T>& L) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) L.m[a][b] = U[(long)(mu * 9 + a * 3 + b) * V + s];
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

template <typename T, int DAG>
__device__ __forceinline__ void all_hops(Spinor<T>& o, const cplx<T>* __restrict__ pin, const cplx<T>* __restrict__ U,
                                         long s, long V, const long* fw, const long* bw) {
  const T sf = DAG ? (T)1 : (T)-1, sb = -sf;
  Spinor<T> p;
  Link<T> L;
#define AMG_HOP4(MU)                                  \
  ld_spinor(pin, fw[MU], V, p); ld_link<T>(U, s, V, MU, L);      hop<T, MU, false>(o, p, L, sf); \
  ld_spinor(pin, bw[MU], V, p); ld_link<T>(U, bw[MU], V, MU, L); hop<T, MU, true>(o, p, L, sb);
  AMG_HOP4(0) AMG_HOP4(1) AMG_HOP4(2) AMG_HOP4(3)
#undef AMG_HOP4
}

Geo4 geo(const int* d);

template <typename T, int DAG, int EPI>
__global__ __launch_bounds__(256) void wilson4d_kernel(WilsonArgs<T> a0, const WilsonArgs<T>* batch) {
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
  const cplx<T>* __restrict__ pin = a.in + ro;
  const cplx<T>* __restrict__ U = a.U;
  const cplx<T>* __restrict__ bvec = a.b;
  cplx<T>* __restrict__ out = a.out;
  cplx<T>* __restrict__ copy_out = a.copy_out;
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
    all_hops<T, DAG>(o, pin, U, s, V, fw, bw);
    if (EPI == EPI_RESID) {
      Spinor<T> b;
      ld_spinor(bvec + ro, s, V, b);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) o.c[sp][k] = csub<T>(b.c[sp][k], o.c[sp][k]);
    }
    st_spinor(out + ro, s, V, o);
    if (copy_out) st_spinor(copy_out + ro, s, V, c);
    if (EPI == EPI_MRDOT || EPI == EPI_NORM) {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const cplx<T> a = o.c[sp][k], r = c.c[sp][k];
          if (EPI == EPI_MRDOT) {
            acc[0] += (double)a.x * r.x + (double)a.y * r.y;
            acc[1] += (double)a.x * r.y - (double)a.y * r.x;
            acc[2] += (double)a.x * a.x + (double)a.y * a.y;
          } else {
            acc[0] += (double)a.x * a.x + (double)a.y * a.y;
          }
        }
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
__global__ __launch_bounds__(256) void wilson4d_split_kernel(double2* __restrict__ out, const double2* __restrict__ in,
                                                             const double2* __restrict__ U, double diag, Geo4 G, long V,
                                                             int b0, int b1, int b2, int b3, int nrhs) {
  const int rhs = blockIdx.y;
  const long ro = (long)rhs * 12 * V;
  const long ks = (long)nrhs * 12 * V;
  const int blk[4] = {b0, b1, b2, b3};
  const double2* __restrict__ pin = in + ro;
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

Geo4 geo(const int* d) {
  Geo4 G;
  long st = 1;
  for (int mu = 0; mu < 4; ++mu) { G.L[mu] = d[mu]; G.st[mu] = st; st *= d[mu]; }
  return G;
}

}  // namespace

template <typename T>
void launch_wilson4d(const WilsonArgs<T>& a, int dagger, int epi, hipStream_t st) {
  const long V = (long)a.L1 * a.L2 * a.L3 * a.L4;
  long nb = (V + 255) / 256;
  if (epi == EPI_MRDOT || epi == EPI_NORM) nb = nb < red_block_cap() ? nb : red_block_cap();
  dim3 grid((unsigned)nb, (unsigned)a.nrhs);
#define AMG_W4(DAG, EPI) dispatch(wilson4d_kernel<T, DAG, EPI>, a, grid, dim3(256), st)
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

void launch_links4d_pack(double2* U64, float2* U32, const double2* canon, long V, hipStream_t st) {
  long nb = (4 * V + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(links4d_pack_kernel, dim3((unsigned)nb), dim3(256), 0, st, U64, U32, canon, V);
}

}  // namespace amg

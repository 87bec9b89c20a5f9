// Two-dimensional U(1) Wilson-Dirac stencil on gfx950.
//
//   (D psi)(x) = (2 + m) psi(x)
//     - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^* psi(x-mu) ]
//
// (operator defined after Eq. (1) of the paper, diagonal read as d + m;
// gamma_1 = sigma_1, gamma_2 = sigma_2).  D^dagger swaps the two projectors.
// Each projector 1 + s gamma_mu (s = +-1) has rank one, so a hop needs one
// complex product:  mu = 1: h = f0 + s f1, result (h, s h);
//                   mu = 2: h = f0 - i s f1, result (h, i s h).
//
// Internal layouts (one thread per site, grid-stride, 16-byte accesses):
//   FP64 spinor: two planes [spin][site] of double2;  links [mu][site] double2
//   FP32 spinor: [site] float4 = (s0, s1);            links [site] float4 = (U_1, U_2)
// These are Layout{V, 2, W} with W = 1 (FP64) and W = 2 (FP32).
#include <cstdlib>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace amg {
namespace {

template <typename T> struct Sp2 { cplx<T> a, b; };

__device__ __forceinline__ Sp2<double> ld2(gptr<const double2> __restrict__ p, long s, long V) {
  return {p[s], p[V + s]};
}
__device__ __forceinline__ Sp2<float> ld2(gptr<const float2> __restrict__ p, long s, long) {
  const float4 q = ((gptr<const float4>)p)[s];
  return {make_float2(q.x, q.y), make_float2(q.z, q.w)};
}
__device__ __forceinline__ void st2(gptr<double2> __restrict__ p, long s, long V, Sp2<double> v) {
  p[s] = v.a; p[V + s] = v.b;
}
__device__ __forceinline__ void st2(gptr<float2> __restrict__ p, long s, long, Sp2<float> v) {
  ((gptr<float4>)p)[s] = make_float4(v.a.x, v.a.y, v.b.x, v.b.y);
}
// streaming (non-temporal) stores for lattices far larger than the caches:
// the result is not read again by this kernel and would only evict the
// neighbour spinors that the other waves still need
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void st2_nt(gptr<double2> __restrict__ p, long s, long V, Sp2<double> v) {
  const v2d a = {v.a.x, v.a.y}, b = {v.b.x, v.b.y};
  __builtin_nontemporal_store(a, (gptr<v2d>)p + s);
  __builtin_nontemporal_store(b, (gptr<v2d>)p + V + s);
}
__device__ __forceinline__ void st2_nt(gptr<float2> __restrict__ p, long s, long, Sp2<float> v) {
  const v4f a = {v.a.x, v.a.y, v.b.x, v.b.y};
  __builtin_nontemporal_store(a, (gptr<v4f>)p + s);
}
// single link U_mu(site)
__device__ __forceinline__ double2 ldU(gptr<const double2> __restrict__ U, long s, long V, int mu) {
  return U[mu * V + s];
}
__device__ __forceinline__ float2 ldU(gptr<const float2> __restrict__ U, long s, long, int mu) {
  return U[2 * s + mu];
}

// The four hops of site s, accumulated as o -= 1/2 (projected, transported neighbour).
// SPLIT: route each hop to out0 (inside the block) or to its own output (crossing a face).
template <typename T, int DAG>
struct Hops {
  long V; int L1, L2;
  __device__ __forceinline__ void neighbours(long s, int& x1, int& x2, long& sp1, long& sm1,
                                             long& sp2, long& sm2) const {
    x1 = (int)(s % L1); x2 = (int)(s / L1);
    sp1 = (x1 == L1 - 1) ? s - (L1 - 1) : s + 1;
    sm1 = (x1 == 0) ? s + (L1 - 1) : s - 1;
    sp2 = (x2 == L2 - 1) ? s - (long)(L2 - 1) * L1 : s + L1;
    sm2 = (x2 == 0) ? s + (long)(L2 - 1) * L1 : s - L1;
  }
  // forward hop in mu = 0 with projector 1 + sg gamma_1 on link u, neighbour f
  static __device__ __forceinline__ Sp2<T> hop1(cplx<T> u, Sp2<T> f, T sg, bool conj_u) {
    const cplx<T> h = mk<T>(f.a.x + sg * f.b.x, f.a.y + sg * f.b.y);
    const cplx<T> uh = conj_u ? cjmul<T>(u, h) : cmul<T>(u, h);
    return {uh, cscale<T>(sg, uh)};
  }
  static __device__ __forceinline__ Sp2<T> hop2(cplx<T> u, Sp2<T> f, T sg, bool conj_u) {
    // h = f0 - i sg f1
    const cplx<T> h = mk<T>(f.a.x + sg * f.b.y, f.a.y - sg * f.b.x);
    const cplx<T> uh = conj_u ? cjmul<T>(u, h) : cmul<T>(u, h);
    return {uh, cscale<T>(sg, ctimesi<T>(uh))};
  }
};

template <typename T>
__device__ __forceinline__ void sub_half(Sp2<T>& o, const Sp2<T>& h) {
  o.a.x -= (T)0.5 * h.a.x; o.a.y -= (T)0.5 * h.a.y;
  o.b.x -= (T)0.5 * h.b.x; o.b.y -= (T)0.5 * h.b.y;
}

template <typename T, int DAG, int EPI, bool NT>
__global__ __launch_bounds__(256) void wilson2d_kernel(WilsonArgs<T> a0, const WilsonArgs<T>* batch) {
  AMG_ARGS(WilsonArgs<T>)
  const int rhs = blockIdx.y;
  const RedArgs& red = a.red;
  if (skip_rhs(red.flags, rhs)) return;
  const int L1 = a.L1, L2 = a.L2;
  const long V = (long)L1 * L2;
  const long ro = (long)rhs * 2 * V;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ U = gl(a.U);
  gptr<const cplx<T>> __restrict__ bvec = gl(a.b);
  gptr<cplx<T>> __restrict__ out = gl(a.out);
  gptr<cplx<T>> __restrict__ copy_out = gl(a.copy_out);
  const T diag = (T)(2.0 + a.mass);
  Hops<T, DAG> H{V, L1, L2};
  const T sf = DAG ? (T)1 : (T)-1;  // forward projector 1 + sf gamma
  const T sb = -sf;
  double acc[3] = {0.0, 0.0, 0.0};
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (long)gridDim.x * blockDim.x) {
    int x1, x2; long sp1, sm1, sp2, sm2;
    H.neighbours(s, x1, x2, sp1, sm1, sp2, sm2);
    const Sp2<T> c = ld2(pin, s, V);
    Sp2<T> o{cscale<T>(diag, c.a), cscale<T>(diag, c.b)};
    sub_half<T>(o, Hops<T, DAG>::hop1(ldU(U, s, V, 0), ld2(pin, sp1, V), sf, false));
    sub_half<T>(o, Hops<T, DAG>::hop1(ldU(U, sm1, V, 0), ld2(pin, sm1, V), sb, true));
    sub_half<T>(o, Hops<T, DAG>::hop2(ldU(U, s, V, 1), ld2(pin, sp2, V), sf, false));
    sub_half<T>(o, Hops<T, DAG>::hop2(ldU(U, sm2, V, 1), ld2(pin, sm2, V), sb, true));
    if (EPI == EPI_RESID) {
      const Sp2<T> bb = ld2(bvec + ro, s, V);
      o = {csub<T>(bb.a, o.a), csub<T>(bb.b, o.b)};
    }
    if (NT) {
      st2_nt(out + ro, s, V, o);
      if (copy_out) st2_nt(copy_out + ro, s, V, c);
    } else {
      st2(out + ro, s, V, o);
      if (copy_out) st2(copy_out + ro, s, V, c);
    }
    if (EPI == EPI_MRDOT) {
      acc[0] += (double)o.a.x * c.a.x + (double)o.a.y * c.a.y + (double)o.b.x * c.b.x + (double)o.b.y * c.b.y;
      acc[1] += (double)o.a.x * c.a.y - (double)o.a.y * c.a.x + (double)o.b.x * c.b.y - (double)o.b.y * c.b.x;
      acc[2] += (double)o.a.x * o.a.x + (double)o.a.y * o.a.y + (double)o.b.x * o.b.x + (double)o.b.y * o.b.y;
    } else if (EPI == EPI_NORM) {
      acc[0] += (double)o.a.x * o.a.x + (double)o.a.y * o.a.y + (double)o.b.x * o.b.x + (double)o.b.y * o.b.y;
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

// ---- x_2-marching form for lattices far larger than the caches -------------
// A wave owns 64 consecutive x_1 sites of a strip of ROWS rows and marches
// along x_2: the x_2 neighbours and the backward x_2 link come from the
// previous row's registers, the x_1 neighbours and the backward x_1 link
// from the adjacent lanes (cross-lane permutes; lanes 0 and 63 load the one
// value outside the wave).  Every spinor and link is then read from HBM once
// (the rows shared with the strips above and below through L2), so the
// loads, like the stores, stream past the caches.  All four epilogues.
__device__ __forceinline__ Sp2<double> ld2_nt(gptr<const double2> __restrict__ p, long s, long V) {
  const v2d a = __builtin_nontemporal_load((gptr<const v2d>)p + s);
  const v2d b = __builtin_nontemporal_load((gptr<const v2d>)p + V + s);
  return {make_double2(a.x, a.y), make_double2(b.x, b.y)};
}
__device__ __forceinline__ Sp2<float> ld2_nt(gptr<const float2> __restrict__ p, long s, long) {
  const v4f q = __builtin_nontemporal_load((gptr<const v4f>)p + s);
  return {make_float2(q.x, q.y), make_float2(q.z, q.w)};
}
// both links of site s: (U_1(s), U_2(s))
__device__ __forceinline__ void ldU12_nt(gptr<const double2> __restrict__ U, long s, long V, double2& u1,
                                         double2& u2) {
  const v2d a = __builtin_nontemporal_load((gptr<const v2d>)U + s);
  const v2d b = __builtin_nontemporal_load((gptr<const v2d>)U + V + s);
  u1 = make_double2(a.x, a.y);
  u2 = make_double2(b.x, b.y);
}
__device__ __forceinline__ void ldU12_nt(gptr<const float2> __restrict__ U, long s, long, float2& u1, float2& u2) {
  const v4f q = __builtin_nontemporal_load((gptr<const v4f>)U + s);
  u1 = make_float2(q.x, q.y);
  u2 = make_float2(q.z, q.w);
}
template <typename T>
__device__ __forceinline__ cplx<T> lane_from(cplx<T> v, int src) {
  return mk<T>(__shfl(v.x, src), __shfl(v.y, src));
}
template <typename T>
__device__ __forceinline__ Sp2<T> lane_from(const Sp2<T>& v, int src) {
  return {lane_from<T>(v.a, src), lane_from<T>(v.b, src)};
}

template <typename T, int DAG, int EPI, int ROWS>
__global__ __launch_bounds__(256) void wilson2d_strip_kernel(WilsonArgs<T> a0, const WilsonArgs<T>* batch) {
  AMG_ARGS(WilsonArgs<T>)
  const int rhs = blockIdx.y;
  const RedArgs& red = a.red;
  if (skip_rhs(red.flags, rhs)) return;  // every block of this rhs: no reduction is started
  const int L1 = a.L1, L2 = a.L2;
  const long V = (long)L1 * L2;
  const long ro = (long)rhs * 2 * V;
  const int lane = threadIdx.x & 63;
  const int nx = L1 >> 6;                                  // tiles along x_1
  const long tiles = (long)nx * (L2 / ROWS);
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ U = gl(a.U);
  gptr<const cplx<T>> __restrict__ bvec = gl(a.b) + ro;
  gptr<cplx<T>> __restrict__ out = gl(a.out) + ro;
  gptr<cplx<T>> __restrict__ copy_out = gl(a.copy_out) + ro;
  const bool copy = a.copy_out != nullptr;
  const T diag = (T)(2.0 + a.mass);
  const T sf = DAG ? (T)1 : (T)-1;  // forward projector 1 + sf gamma
  const T sb = -sf;
  const int left = (lane + 63) & 63, right = (lane + 1) & 63;
  double acc[3] = {0.0, 0.0, 0.0};
  auto strip = [&](int tile) {
    const int tx = tile % nx, ty = tile / nx;
    const int x1 = tx * 64 + lane;
    const int x1m = (x1 == 0) ? L1 - 1 : x1 - 1;
    const int x1p = (x1 == L1 - 1) ? 0 : x1 + 1;
    const int y0 = ty * ROWS, yl = y0 + ROWS - 1;
    // The rows a strip shares with its neighbours (the row below it, its
    // first and last rows, the row above it) and the links of its last row
    // are read at the start, through the caches: adjacent strips start at
    // about the same time on the same XCD, so the second reader of a shared
    // row finds it in L2.  The rows in between stream.
    const long sm0 = (long)((y0 == 0) ? L2 - 1 : y0 - 1) * L1 + x1;
    const long sl = (long)yl * L1 + x1;
    const long sh = (long)((yl == L2 - 1) ? 0 : yl + 1) * L1 + x1;
    Sp2<T> cm = ld2(pin, sm0, V);
    cplx<T> u2m = ldU(U, sm0, V, 1);
    Sp2<T> cc = ld2(pin, (long)y0 * L1 + x1, V);
    const Sp2<T> c_last = ld2(pin, sl, V), c_above = ld2(pin, sh, V);
    const cplx<T> u1_last = ldU(U, sl, V, 0), u2_last = ldU(U, sl, V, 1);
#pragma unroll (ROWS <= 4 ? ROWS : 2)
    for (int t = 0; t < ROWS; ++t) {
      const int y = y0 + t;
      const long s = (long)y * L1 + x1;
      const long sn = s + L1;  // used for t <= ROWS - 3 only: y + 1 < yl, no wrap
      const Sp2<T> cn = (t == ROWS - 1) ? c_above : (t == ROWS - 2) ? c_last : ld2_nt(pin, sn, V);
      cplx<T> u1 = u1_last, u2 = u2_last;
      if (t < ROWS - 1) ldU12_nt(U, s, V, u1, u2);
      Sp2<T> cl = lane_from<T>(cc, left), cr = lane_from<T>(cc, right);
      cplx<T> u1l = lane_from<T>(u1, left);
      if (lane == 0) {
        cl = ld2(pin, (long)y * L1 + x1m, V);
        u1l = ldU(U, (long)y * L1 + x1m, V, 0);
      }
      if (lane == 63) cr = ld2(pin, (long)y * L1 + x1p, V);
      Sp2<T> o{cscale<T>(diag, cc.a), cscale<T>(diag, cc.b)};
      sub_half<T>(o, Hops<T, DAG>::hop1(u1, cr, sf, false));
      sub_half<T>(o, Hops<T, DAG>::hop1(u1l, cl, sb, true));
      sub_half<T>(o, Hops<T, DAG>::hop2(u2, cn, sf, false));
      sub_half<T>(o, Hops<T, DAG>::hop2(u2m, cm, sb, true));
      if (EPI == EPI_RESID) {
        const Sp2<T> bb = ld2_nt(bvec, s, V);
        o = {csub<T>(bb.a, o.a), csub<T>(bb.b, o.b)};
      }
      st2_nt(out, s, V, o);
      if (copy) st2_nt(copy_out, s, V, cc);
      if (EPI == EPI_MRDOT) {
        acc[0] += (double)o.a.x * cc.a.x + (double)o.a.y * cc.a.y + (double)o.b.x * cc.b.x + (double)o.b.y * cc.b.y;
        acc[1] += (double)o.a.x * cc.a.y - (double)o.a.y * cc.a.x + (double)o.b.x * cc.b.y - (double)o.b.y * cc.b.x;
        acc[2] += (double)o.a.x * o.a.x + (double)o.a.y * o.a.y + (double)o.b.x * o.b.x + (double)o.b.y * o.b.y;
      } else if (EPI == EPI_NORM) {
        acc[0] += (double)o.a.x * o.a.x + (double)o.a.y * o.a.y + (double)o.b.x * o.b.x + (double)o.b.y * o.b.y;
      }
      cm = cc;
      cc = cn;
      u2m = u2;
    }
  };
  // one tile per wave: the waves of a pass cover consecutive tiles, so
  // adjacent strips run at the same time
  const int tile0 = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (EPI == EPI_PLAIN || EPI == EPI_RESID) {  // a wave for every tile, no reduction
    if (tile0 < tiles) strip(tile0);
    return;
  }
  // reducing epilogues: capped grid, tile stride
  for (long tile = tile0; tile < tiles; tile += (long)gridDim.x * 4) strip((int)tile);
  if (EPI == EPI_MRDOT) {
    double tot[3];
    if (grid_reduce<3>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) finalize_mr(tot, red, rhs);
  } else if (EPI == EPI_NORM) {
    double a1[1] = {acc[0]}, tot[1];
    if (grid_reduce<1>(a1, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) red.scal[red.slot + rhs] = tot[0];
  }
}

// Split apply for the Galerkin product: out[k] (k = 0..4) for every input
// field; out[0] = diagonal + hops that stay inside the block, out[1 + dir] =
// the hop in direction dir (0:+1, 1:-1, 2:+2, 3:-2) when it leaves the block
// through its face.  FP64, layout W = 1.
__global__ __launch_bounds__(256) void wilson2d_split_kernel(
    double2* __restrict__ out_, const double2* __restrict__ in, const double2* __restrict__ U_,
    double diag, int L1, int L2, int b1, int b2, int nrhs) {
  const int rhs = blockIdx.y;
  const long V = (long)L1 * L2;
  const long ro = (long)rhs * 2 * V;
  const long ostride = (long)nrhs * 2 * V;  // between output kinds
  gptr<const double2> __restrict__ pin = gl(in) + ro;
  gptr<const double2> __restrict__ U = gl(U_);
  gptr<double2> __restrict__ out = gl(out_);
  Hops<double, 0> H{V, L1, L2};
  for (long s = (long)blockIdx.x * blockDim.x + threadIdx.x; s < V; s += (long)gridDim.x * blockDim.x) {
    int x1, x2; long sp1, sm1, sp2, sm2;
    H.neighbours(s, x1, x2, sp1, sm1, sp2, sm2);
    const Sp2<double> c = ld2(pin, s, V);
    Sp2<double> o0{cscale<double>(diag, c.a), cscale<double>(diag, c.b)};
    Sp2<double> hop[4];
    Sp2<double> z{mk<double>(0, 0), mk<double>(0, 0)};
    for (int k = 0; k < 4; ++k) hop[k] = z;
    Sp2<double> t;
    t = z; sub_half<double>(t, Hops<double, 0>::hop1(ldU(U, s, V, 0), ld2(pin, sp1, V), -1.0, false));
    if (x1 % b1 == b1 - 1) hop[0] = t; else { o0.a = cadd<double>(o0.a, t.a); o0.b = cadd<double>(o0.b, t.b); }
    t = z; sub_half<double>(t, Hops<double, 0>::hop1(ldU(U, sm1, V, 0), ld2(pin, sm1, V), 1.0, true));
    if (x1 % b1 == 0) hop[1] = t; else { o0.a = cadd<double>(o0.a, t.a); o0.b = cadd<double>(o0.b, t.b); }
    t = z; sub_half<double>(t, Hops<double, 0>::hop2(ldU(U, s, V, 1), ld2(pin, sp2, V), -1.0, false));
    if (x2 % b2 == b2 - 1) hop[2] = t; else { o0.a = cadd<double>(o0.a, t.a); o0.b = cadd<double>(o0.b, t.b); }
    t = z; sub_half<double>(t, Hops<double, 0>::hop2(ldU(U, sm2, V, 1), ld2(pin, sm2, V), 1.0, true));
    if (x2 % b2 == 0) hop[3] = t; else { o0.a = cadd<double>(o0.a, t.a); o0.b = cadd<double>(o0.b, t.b); }
    st2(out + ro, s, V, o0);
    for (int k = 0; k < 4; ++k) st2(out + (k + 1) * ostride + ro, s, V, hop[k]);
  }
}

}  // namespace

// lattices from this many sites on stream their results past the caches
constexpr long kStreamSites = 1L << 20;

template <typename T>
void launch_wilson2d(const WilsonArgs<T>& a, int dagger, int epi, hipStream_t st) {
  const long V = (long)a.L1 * a.L2;
  long nb = (V + 255) / 256;
  if (epi == EPI_MRDOT || epi == EPI_NORM) nb = nb < red_block_cap() ? nb : red_block_cap();
  dim3 grid((unsigned)nb, (unsigned)a.nrhs);
#define AMG_W2N(DAG, EPI, NT) dispatch(wilson2d_kernel<T, DAG, EPI, NT>, a, grid, dim3(256), st)
#define AMG_W2(DAG, EPI) if (nt) { AMG_W2N(DAG, EPI, true); } else { AMG_W2N(DAG, EPI, false); }
  static const bool nt_on = [] {
    const char* e = std::getenv("AMG_STREAM_STORES");
    return e ? std::atoi(e) != 0 : true;
  }();
  const bool nt = nt_on && V >= kStreamSites;
  // rows per strip of the x_2-marching kernel (0: one site per thread);
  // measured best at 4096^2: 4 in FP64 (72 % of 8 TB/s), 2 in FP32 (77 %)
  static const int strip_rows = [] {
    const char* e = std::getenv("AMG_W2_STRIP");
    return e ? std::atoi(e) : (sizeof(T) == 8 ? 4 : 2);
  }();
  // (not while recording for a batch: every instance must record the same kernels)
  if ((strip_rows == 2 || strip_rows == 4 || strip_rows == 8 || strip_rows == 16) && nt &&
      current_recorder() == nullptr && a.L1 % 64 == 0 && a.L2 % strip_rows == 0) {
    const long tiles = (long)(a.L1 / 64) * (a.L2 / strip_rows);
    long nbs = (tiles + 3) / 4;
    if (epi == EPI_MRDOT || epi == EPI_NORM) nbs = nbs < red_block_cap() ? nbs : red_block_cap();
    const dim3 gs((unsigned)nbs, (unsigned)a.nrhs);
#define AMG_W2S(DAG, EPI, R) dispatch(wilson2d_strip_kernel<T, DAG, EPI, R>, a, gs, dim3(256), st)
#define AMG_W2SR(DAG, EPI)                                     \
    switch (strip_rows) {                                      \
      case 2: AMG_W2S(DAG, EPI, 2); break;                     \
      case 4: AMG_W2S(DAG, EPI, 4); break;                     \
      case 8: AMG_W2S(DAG, EPI, 8); break;                     \
      default: AMG_W2S(DAG, EPI, 16); break;                   \
    }
#define AMG_W2SE(EPI) if (dagger) { AMG_W2SR(1, EPI) } else { AMG_W2SR(0, EPI) }
    switch (epi) {
      case EPI_PLAIN: AMG_W2SE(EPI_PLAIN) break;
      case EPI_RESID: AMG_W2SE(EPI_RESID) break;
      case EPI_MRDOT: AMG_W2SE(EPI_MRDOT) break;
      default: AMG_W2SE(EPI_NORM) break;
    }
#undef AMG_W2SE
#undef AMG_W2SR
#undef AMG_W2S
    return;
  }
  if (dagger) {
    switch (epi) {
      case EPI_PLAIN: AMG_W2(1, EPI_PLAIN); break;
      case EPI_MRDOT: AMG_W2(1, EPI_MRDOT); break;
      case EPI_RESID: AMG_W2(1, EPI_RESID); break;
      default: AMG_W2(1, EPI_NORM); break;
    }
  } else {
    switch (epi) {
      case EPI_PLAIN: AMG_W2(0, EPI_PLAIN); break;
      case EPI_MRDOT: AMG_W2(0, EPI_MRDOT); break;
      case EPI_RESID: AMG_W2(0, EPI_RESID); break;
      default: AMG_W2(0, EPI_NORM); break;
    }
  }
#undef AMG_W2N
#undef AMG_W2
}

template void launch_wilson2d<double>(const WilsonArgs<double>&, int, int, hipStream_t);
template void launch_wilson2d<float>(const WilsonArgs<float>&, int, int, hipStream_t);

void launch_wilson2d_split(double2* out, const double2* in, const double2* U, double mass, int L1,
                           int L2, int b1, int b2, int nrhs, hipStream_t st) {
  const long V = (long)L1 * L2;
  dim3 grid((unsigned)((V + 255) / 256), (unsigned)nrhs);
  hipLaunchKernelGGL(wilson2d_split_kernel, grid, dim3(256), 0, st, out, in, U, 2.0 + mass, L1, L2,
                     b1, b2, nrhs);
}

}  // namespace amg

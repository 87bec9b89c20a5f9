// Vector kernels of the smoother and the Krylov solvers: MR updates, GCR
// orthogonalisation / updates, CG on the normal equations, norms, and the
// precision / layout conversions.  All coefficients stay on the device
// (written by the last block of the producing reduction, read by the
// consumers), so a solver step needs no host round trip.
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

#include <cstring>

namespace amg {
namespace {

inline unsigned nblocks(long n, long cap) {
  long b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// grid of a reducing kernel: ept elements per thread (more blocks keep more
// loads in flight, fewer leave fewer partial sums for the last block), at
// most the reduction cap
inline int red_ept() {
  static int e = [] {
    const char* v = std::getenv("AMG_RED_EPT");
    return v ? std::max(1, std::atoi(v)) : 1;
  }();
  return e;
}
inline unsigned red_blocks(long n) {
  const long per = 256L * red_ept();
  long b = (n + per - 1) / per;
  if (b > red_block_cap()) b = red_block_cap();
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define GRID_STRIDE(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

template <typename Tin, typename Tout>
struct CvArgs {
  cplx<Tout>* out;
  const cplx<Tin>* in;
  Layout li, lo;
  int nrhs;
};
template <typename Tin, typename Tout>
__global__ void convert_kernel(CvArgs<Tin, Tout> a0, const CvArgs<Tin, Tout>* batch) {
  AMG_ARGS(CvArgs<Tin, Tout>)
  const auto pin = gl(a.in);
  const auto pout = gl(a.out);
  const long n = a.li.per_rhs();
  const long ro = (long)blockIdx.y * n;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / a.li.V);
    const long s = i - (long)c * a.li.V;
    const cplx<Tin> z = pin[ro + a.li.off(s, c)];
    pout[ro + a.lo.off(s, c)] = mk<Tout>((Tout)z.x, (Tout)z.y);
  }
}

// dst = src (src == nullptr: dst = 0), n complex per rhs
template <typename T>
struct FillArgs {
  cplx<T>* dst;
  const cplx<T>* src;
  long n;
  int nrhs;
};
template <typename T>
__global__ void fill_kernel(FillArgs<T> a0, const FillArgs<T>* batch) {
  AMG_ARGS(FillArgs<T>)
  const auto dst = gl(a.dst);
  const auto src = gl(a.src);
  const long ro = (long)blockIdx.y * a.n;
  GRID_STRIDE(i, a.n) {
    cplx<T> v = mk<T>(0, 0);
    if (a.src) v = src[ro + i];
    dst[ro + i] = v;
  }
}

__global__ void p_to_f32_kernel(float2* __restrict__ out, const double2* __restrict__ in, long n) {
  GRID_STRIDE(i, n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ void p_to_bf16_kernel(bf16x2* __restrict__ out, const double2* __restrict__ in, long n) {
  GRID_STRIDE(i, n) out[i] = bf16x2{f2bf((float)in[i].x), f2bf((float)in[i].y)};
}
__global__ void p_roundtrip_bf16_kernel(double2* __restrict__ P, long n) {
  GRID_STRIDE(i, n) {
    const double2 z = P[i];
    P[i] = make_double2((double)bf2f(f2bf((float)z.x)), (double)bf2f(f2bf((float)z.y)));
  }
}

template <typename T>
struct MrArgs {
  cplx<T>* x;
  cplx<T>* r_out;
  const cplx<T>* r_in;
  const cplx<T>* p;
  const double* alpha;  // [2 rhs] (re, im), or nullptr: from the partial sums below
  long n;
  int first, update_r;
  const int* flags;
  int nrhs;
  const double* part;   // per-block <p, r> (re, im), <p, p> of the stencil launch (EPI_MRPART)
  int nblk;             // its number of blocks
  double omega;
};
template <typename T>
__global__ void mr_update_kernel(MrArgs<T> a0, const MrArgs<T>* batch) {
  AMG_ARGS(MrArgs<T>)
  const int rhs = blockIdx.y;
  if (skip_rhs(a.flags, rhs)) return;
  cplx<T> al;
  if (a.alpha != nullptr) {
    al = mk<T>((T)gl(a.alpha)[2 * rhs], (T)gl(a.alpha)[2 * rhs + 1]);
  } else {
    // alpha = omega <p, r> / <p, p> from the stencil's per-block sums
    double tot[3];
    sum_partials<3>(a.part, a.nblk, rhs, tot);
    const double s = tot[2] > 0.0 ? a.omega / tot[2] : 0.0;
    al = mk<T>((T)(s * tot[0]), (T)(s * tot[1]));
  }
  const long ro = (long)rhs * a.n;
  if (sizeof(T) == 4 && (a.n & 1) == 0) {
    // FP32: two complex numbers per 16-byte access
    using V4 = float4;
    const long n2 = a.n / 2, ro2 = ro / 2;
    gptr<const V4> __restrict__ rin = (gptr<const V4>)a.r_in + ro2;
    gptr<const V4> __restrict__ pp = (gptr<const V4>)a.p + ro2;
    gptr<V4> __restrict__ xx = (gptr<V4>)a.x + ro2;
    gptr<V4> __restrict__ rout = (gptr<V4>)a.r_out + ro2;
    const float ar = (float)al.x, ai = (float)al.y;
    GRID_STRIDE(i, n2) {
      const V4 r = rin[i];
      V4 x = a.first ? make_float4(0.f, 0.f, 0.f, 0.f) : xx[i];
      x.x += ar * r.x - ai * r.y; x.y += ar * r.y + ai * r.x;
      x.z += ar * r.z - ai * r.w; x.w += ar * r.w + ai * r.z;
      xx[i] = x;
      if (a.update_r) {
        const V4 q = pp[i];
        rout[i] = make_float4(r.x - (ar * q.x - ai * q.y), r.y - (ar * q.y + ai * q.x),
                              r.z - (ar * q.z - ai * q.w), r.w - (ar * q.w + ai * q.z));
      }
    }
    return;
  }
  const auto r_in = gl(a.r_in);
  const auto x = gl(a.x), r_out = gl(a.r_out);
  const auto p = gl(a.p);
  GRID_STRIDE(i, a.n) {
    const cplx<T> r = r_in[ro + i];
    const cplx<T> ar = cmul<T>(al, r);
    x[ro + i] = a.first ? ar : cadd<T>(x[ro + i], ar);
    if (a.update_r) r_out[ro + i] = csub<T>(r, cmul<T>(al, p[ro + i]));
  }
}

template <typename T>
struct NormArgs {
  const cplx<T>* v;
  long n;
  RedArgs red;
  int nrhs;
};
template <typename T>
__global__ __launch_bounds__(256) void norm2_kernel(NormArgs<T> a0, const NormArgs<T>* batch) {
  AMG_ARGS(NormArgs<T>)
  const auto v = gl(a.v);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  double acc[1] = {0.0};
  GRID_STRIDE(i, a.n) { const cplx<T> z = v[ro + i]; acc[0] += (double)z.x * z.x + (double)z.y * z.y; }
  double tot[1];
  if (grid_reduce<1>(acc, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) scal[a.red.slot + rhs] = tot[0];
}

// arguments shared by the GCR step kernels; directions W_j = Wb + j * dstride
template <typename T>
struct GcrArgs {
  cplx<T>* x;
  cplx<T>* r;
  cplx<T>* w;        // current direction (W_k)
  cplx<T>* z;        // current preconditioned direction (Z_k)
  const cplx<T>* zsrc;
  cplx<T>* Wb;
  cplx<T>* Zb;
  long dstride, n;
  int k;
  RedArgs red;
  int beta_slot, ww_slot, alpha_slot, rr_slot, bb_slot;
  double tol2;
  int* set_flags;
  int nrhs;
};

// beta_j = <W_j, w> / <W_j, W_j>, j < k  (classical Gram-Schmidt coefficients)
template <typename T, int KM>
__global__ __launch_bounds__(256) void gcr_mdot_kernel(GcrArgs<T> a0, const GcrArgs<T>* batch) {
  AMG_ARGS(GcrArgs<T>)
  const auto w = gl(a.w), Wb = gl(a.Wb);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  const int k = a.k;
  double acc[2 * KM];
#pragma unroll
  for (int j = 0; j < 2 * KM; ++j) acc[j] = 0.0;
  GRID_STRIDE(i, a.n) {
    const cplx<T> wi = w[ro + i];
    // every load is issued (clamped to a stored direction), the surplus ones
    // are masked: no branch between the loads, so they are all in flight
    cplx<T> q[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) q[j] = Wb[(long)(j < k ? j : k - 1) * a.dstride + ro + i];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      const double m = j < k ? 1.0 : 0.0;
      acc[2 * j] += m * ((double)q[j].x * wi.x + (double)q[j].y * wi.y);
      acc[2 * j + 1] += m * ((double)q[j].x * wi.y - (double)q[j].y * wi.x);
    }
  }
  double tot[2 * KM];
  if (grid_reduce<2 * KM>(acc, a.red.part, a.red.ticket, rhs, tot, 2 * k, 2 * KM) && threadIdx.x == 0) {
    for (int j = 0; j < k; ++j) {
      const double ww = scal[a.ww_slot + rhs * GCR_KMAX + j];
      const double s = ww > 0.0 ? 1.0 / ww : 0.0;
      scal[a.beta_slot + (rhs * GCR_KMAX + j) * 2] = tot[2 * j] * s;
      scal[a.beta_slot + (rhs * GCR_KMAX + j) * 2 + 1] = tot[2 * j + 1] * s;
    }
  }
}

// w -= sum_j beta_j W_j ; z -= sum_j beta_j Z_j ; then <w,w> and alpha = <w,r>/<w,w>
template <typename T, int KM>
__global__ __launch_bounds__(256) void gcr_maxpy_kernel(GcrArgs<T> a0, const GcrArgs<T>* batch) {
  AMG_ARGS(GcrArgs<T>)
  const auto w = gl(a.w), z = gl(a.z), Wb = gl(a.Wb), Zb = gl(a.Zb);
  const auto r = gl(a.r);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  const int k = a.k;
  const auto beta = scal + a.beta_slot + (long)rhs * GCR_KMAX * 2;
  cplx<T> b[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j)
    b[j] = j < k ? mk<T>((T)beta[2 * j], (T)beta[2 * j + 1]) : mk<T>(0, 0);
  double acc[3] = {0.0, 0.0, 0.0};
  GRID_STRIDE(i, a.n) {
    cplx<T> wi = w[ro + i];
    cplx<T> zi = z[ro + i];
    if (k > 0) {
      cplx<T> wq[KM], zq[KM];
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        const long off = (long)(j < k ? j : k - 1) * a.dstride + ro + i;
        wq[j] = Wb[off];
        zq[j] = Zb[off];
      }
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        wi = csub<T>(wi, cmul<T>(b[j], wq[j]));
        zi = csub<T>(zi, cmul<T>(b[j], zq[j]));
      }
    }
    if (k > 0) { w[ro + i] = wi; z[ro + i] = zi; }
    const cplx<T> ri = r[ro + i];
    acc[0] += (double)wi.x * wi.x + (double)wi.y * wi.y;
    acc[1] += (double)wi.x * ri.x + (double)wi.y * ri.y;
    acc[2] += (double)wi.x * ri.y - (double)wi.y * ri.x;
  }
  double tot[3];
  if (grid_reduce<3>(acc, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) {
    const double ww = tot[0];
    scal[a.ww_slot + rhs * GCR_KMAX + k] = ww;
    const double s = ww > 0.0 ? 1.0 / ww : 0.0;
    scal[a.alpha_slot + 2 * rhs] = tot[1] * s;
    scal[a.alpha_slot + 2 * rhs + 1] = tot[2] * s;
  }
}

// x += alpha z ; r -= alpha w ; rr = <r,r> ; optionally flag rr <= tol2 * bb
template <typename T>
__global__ __launch_bounds__(256) void gcr_update_kernel(GcrArgs<T> a0, const GcrArgs<T>* batch) {
  AMG_ARGS(GcrArgs<T>)
  const auto x = gl(a.x), z = gl(a.z), r = gl(a.r), w = gl(a.w);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  const cplx<T> al = mk<T>((T)scal[a.alpha_slot + 2 * rhs], (T)scal[a.alpha_slot + 2 * rhs + 1]);
  double acc[1] = {0.0};
  GRID_STRIDE(i, a.n) {
    x[ro + i] = cadd<T>(x[ro + i], cmul<T>(al, z[ro + i]));
    const cplx<T> ri = csub<T>(r[ro + i], cmul<T>(al, w[ro + i]));
    r[ro + i] = ri;
    acc[0] += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  double tot[1];
  if (grid_reduce<1>(acc, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) {
    scal[a.rr_slot + rhs] = tot[0];
    if (a.set_flags) gl(a.set_flags)[rhs] = (tot[0] <= a.tol2 * scal[a.bb_slot + rhs]) ? 1 : 0;
  }
}

// GCR step, part 2 of the fused variant: w' = w - sum_j beta_j W_j,
// z' = zsrc - sum_j beta_j Z_j (stored as direction k), x += alpha z',
// r -= alpha w', <r, r> and flags.
// RED = false: no <r, r> (the next step's dots kernel takes it).
template <typename T, int KM, bool RED>
__global__ __launch_bounds__(256) void gcr_update2_kernel(GcrArgs<T> a0, const GcrArgs<T>* batch) {
  AMG_ARGS(GcrArgs<T>)
  const auto x = gl(a.x), r = gl(a.r), Wb = gl(a.Wb), Zb = gl(a.Zb);
  const auto zsrc = gl(a.zsrc);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  const int k = a.k;
  const auto beta = scal + a.beta_slot + (long)rhs * GCR_KMAX * 2;
  const cplx<T> al = mk<T>((T)scal[a.alpha_slot + 2 * rhs], (T)scal[a.alpha_slot + 2 * rhs + 1]);
  const auto Wk = Wb + (long)k * a.dstride + ro;
  const auto Zk = Zb + (long)k * a.dstride + ro;
  // coefficients in registers (zero past k); every direction load is issued
  // (clamped to a stored one), so they are all in flight at once
  cplx<T> bj[KM > 0 ? KM : 1];
#pragma unroll
  for (int j = 0; j < KM; ++j) bj[j] = j < k ? mk<T>((T)beta[2 * j], (T)beta[2 * j + 1]) : mk<T>(0, 0);
  double acc[1] = {0.0};
  GRID_STRIDE(i, a.n) {
    cplx<T> wi = Wk[i], zi = zsrc[ro + i];
    if (KM > 0) {
      cplx<T> wq[KM > 0 ? KM : 1], zq[KM > 0 ? KM : 1];
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        const long off = (long)(j < k ? j : k - 1) * a.dstride + ro + i;
        wq[j] = Wb[off];
        zq[j] = Zb[off];
      }
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        wi = csub<T>(wi, cmul<T>(bj[j], wq[j]));
        zi = csub<T>(zi, cmul<T>(bj[j], zq[j]));
      }
    }
    Wk[i] = wi;
    Zk[i] = zi;
    x[ro + i] = cadd<T>(x[ro + i], cmul<T>(al, zi));
    const cplx<T> ri = csub<T>(r[ro + i], cmul<T>(al, wi));
    r[ro + i] = ri;
    if (RED) acc[0] += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  if (!RED) return;
  double tot[1];
  if (grid_reduce<1>(acc, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) {
    scal[a.rr_slot + rhs] = tot[0];
    if (a.set_flags) gl(a.set_flags)[rhs] = (tot[0] <= a.tol2 * scal[a.bb_slot + rhs]) ? 1 : 0;
  }
}

// flags[rhs] = inherit[rhs] || scal[rr] <= tol2 * scal[bb]   (one block, thread per rhs)
struct FlagArgs {
  int* flags;
  const int* inherit;
  const double* scal;
  int rr_slot, bb_slot;
  double tol2;
  int nrhs;
};
__global__ void set_flags_kernel(FlagArgs a0, const FlagArgs* batch) {
  AMG_PICK(a, FlagArgs)
  const int rhs = threadIdx.x;
  if (rhs < a.nrhs)
    a.flags[rhs] = ((a.inherit && a.inherit[rhs]) || a.scal[a.rr_slot + rhs] <= a.tol2 * a.scal[a.bb_slot + rhs]) ? 1 : 0;
}

// out[rhs] = scal[slot + rhs] (collects scalars of many instances in one array)
struct GatherArgs {
  double* out;
  const double* scal;
  int slot;
  int nrhs;
};
__global__ void gather_kernel(GatherArgs a0, const GatherArgs* batch) {
  AMG_PICK(a, GatherArgs)
  const int rhs = threadIdx.x;
  if (rhs < a.nrhs) a.out[rhs] = a.scal[a.slot + rhs];
}

// GCR step with one reduction for the orthogonalisation: the sums
// c_j = <W_j, w> (j < k), <w, w> and <w, r> in one pass; the last block forms
// beta_j = c_j / <W_j, W_j>, the norm of the orthogonalised direction
// <w', w'> = <w, w> - sum_j |c_j|^2 / <W_j, W_j> (the stored W_j are mutually
// orthogonal) and alpha = <w', r> / <w', w'> with <w', r> = <w, r> (r is
// orthogonal to every stored W_j).  gcr_update2 then applies the step.
// RR: also <r, r> of the current residual (the previous step's result) into
// the rr slot, and the convergence flag rr <= tol2 * bb — the stopping test
// of the previous step, taken here so that the update needs no reduction.
template <typename T, int KM, bool RR>
__global__ __launch_bounds__(256) void gcr_dots_kernel(GcrArgs<T> a0, const GcrArgs<T>* batch) {
  AMG_ARGS(GcrArgs<T>)
  const auto w = gl(a.w), Wb = gl(a.Wb), r = gl(a.r);
  const auto scal = gl(a.red.scal);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long ro = (long)rhs * a.n;
  const int k = a.k;
  constexpr int NV = 2 * KM + 3 + (RR ? 1 : 0);
  // the scalars the last block needs, loaded now (their latency overlaps the sums)
  double wwj[KM > 0 ? KM : 1], bbv = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < KM; ++j) wwj[j] = scal[a.ww_slot + rhs * GCR_KMAX + (j < k ? j : 0)];
    if (RR) bbv = scal[a.bb_slot + rhs];
  }
  double acc[NV];
#pragma unroll
  for (int j = 0; j < NV; ++j) acc[j] = 0.0;
  GRID_STRIDE(i, a.n) {
    const cplx<T> wi = w[ro + i], ri = r[ro + i];
    if (KM > 0) {
      // clamped loads (no branch between them), surplus terms masked
      cplx<T> q[KM > 0 ? KM : 1];
#pragma unroll
      for (int j = 0; j < KM; ++j) q[j] = Wb[(long)(j < k ? j : k - 1) * a.dstride + ro + i];
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        const double m = j < k ? 1.0 : 0.0;
        acc[2 * j] += m * ((double)q[j].x * wi.x + (double)q[j].y * wi.y);
        acc[2 * j + 1] += m * ((double)q[j].x * wi.y - (double)q[j].y * wi.x);
      }
    }
    acc[2 * KM] += (double)wi.x * wi.x + (double)wi.y * wi.y;
    acc[2 * KM + 1] += (double)wi.x * ri.x + (double)wi.y * ri.y;
    acc[2 * KM + 2] += (double)wi.x * ri.y - (double)wi.y * ri.x;
    if (RR) acc[NV - 1] += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  double tot[NV];
  // slots of directions j >= k are zero
  if (grid_reduce<NV>(acc, a.red.part, a.red.ticket, rhs, tot, 2 * k, 2 * KM) && threadIdx.x == 0) {
    double wwp = tot[2 * KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j >= k) break;
      const double s = wwj[j] > 0.0 ? 1.0 / wwj[j] : 0.0;
      const double cr = tot[2 * j], ci = tot[2 * j + 1];
      scal[a.beta_slot + (rhs * GCR_KMAX + j) * 2] = cr * s;
      scal[a.beta_slot + (rhs * GCR_KMAX + j) * 2 + 1] = ci * s;
      wwp -= (cr * cr + ci * ci) * s;
    }
    if (RR) {
      scal[a.rr_slot + rhs] = tot[NV - 1];
      if (a.set_flags) gl(a.set_flags)[rhs] = (tot[NV - 1] <= a.tol2 * bbv) ? 1 : 0;
    }
    scal[a.ww_slot + rhs * GCR_KMAX + k] = wwp;
    const double s = wwp > 0.0 ? 1.0 / wwp : 0.0;
    scal[a.alpha_slot + 2 * rhs] = tot[2 * KM + 1] * s;
    scal[a.alpha_slot + 2 * rhs + 1] = tot[2 * KM + 2] * s;
  }
}

__global__ __launch_bounds__(256) void cg_update_kernel(double2* __restrict__ x, double2* __restrict__ r,
                                                        const double2* __restrict__ p, const double2* __restrict__ q,
                                                        long n, RedArgs red, int gamma_slot, int qq_slot, int rr_slot) {
  const int rhs = blockIdx.y;
  const long ro = (long)rhs * n;
  const double qq = red.scal[qq_slot + rhs];
  const double a = qq > 0.0 ? red.scal[gamma_slot + rhs] / qq : 0.0;
  double acc[1] = {0.0};
  GRID_STRIDE(i, n) {
    const double2 pi = p[ro + i], qi = q[ro + i];
    double2 xi = x[ro + i], ri = r[ro + i];
    xi.x += a * pi.x; xi.y += a * pi.y;
    ri.x -= a * qi.x; ri.y -= a * qi.y;
    x[ro + i] = xi; r[ro + i] = ri;
    acc[0] += ri.x * ri.x + ri.y * ri.y;
  }
  double tot[1];
  if (grid_reduce<1>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) red.scal[rr_slot + rhs] = tot[0];
}

__global__ void cg_pupdate_kernel(double2* __restrict__ p, const double2* __restrict__ s, long n, const double* scal,
                                  int gnew_slot, int gold_slot) {
  const int rhs = blockIdx.y;
  const long ro = (long)rhs * n;
  const double go = scal[gold_slot + rhs];
  const double b = go > 0.0 ? scal[gnew_slot + rhs] / go : 0.0;
  GRID_STRIDE(i, n) {
    const double2 si = s[ro + i];
    double2 pi = p[ro + i];
    pi.x = si.x + b * pi.x; pi.y = si.y + b * pi.y;
    p[ro + i] = pi;
  }
}

}  // namespace

template <typename Tin, typename Tout>
void launch_convert(cplx<Tout>* out, const cplx<Tin>* in, long V, int dof, int Win, int Wout, int nrhs, hipStream_t st) {
  CvArgs<Tin, Tout> a{out, in, Layout{V, dof, Win}, Layout{V, dof, Wout}, nrhs};
  dispatch(convert_kernel<Tin, Tout>, a, dim3(nblocks(V * dof, 1L << 20), (unsigned)nrhs), dim3(256), st);
}
template void launch_convert<double, double>(double2*, const double2*, long, int, int, int, int, hipStream_t);
template void launch_convert<double, float>(float2*, const double2*, long, int, int, int, int, hipStream_t);
template void launch_convert<float, double>(double2*, const float2*, long, int, int, int, int, hipStream_t);
template void launch_convert<float, float>(float2*, const float2*, long, int, int, int, int, hipStream_t);

template <typename T>
void launch_fill(cplx<T>* dst, const cplx<T>* src, long n, int nrhs, hipStream_t st) {
  FillArgs<T> a{dst, src, n, nrhs};
  dispatch(fill_kernel<T>, a, dim3(nblocks(n, 1L << 20), (unsigned)nrhs), dim3(256), st);
}
template void launch_fill<double>(double2*, const double2*, long, int, hipStream_t);
template void launch_fill<float>(float2*, const float2*, long, int, hipStream_t);

void launch_p_convert(void* out, int pkind, const double2* in, long n, hipStream_t st) {
  if (pkind == P_F32)
    hipLaunchKernelGGL(p_to_f32_kernel, dim3(nblocks(n, 1L << 20)), dim3(256), 0, st, (float2*)out, in, n);
  else if (pkind == P_BF16)
    hipLaunchKernelGGL(p_to_bf16_kernel, dim3(nblocks(n, 1L << 20)), dim3(256), 0, st, (bf16x2*)out, in, n);
}

void launch_p_roundtrip_bf16(double2* P, long n, hipStream_t st) {
  hipLaunchKernelGGL(p_roundtrip_bf16_kernel, dim3(nblocks(n, 1L << 20)), dim3(256), 0, st, P, n);
}

template <typename T>
void launch_mr_update(cplx<T>* x, cplx<T>* r_out, const cplx<T>* r_in, const cplx<T>* p, const double* alpha, long n,
                      int nrhs, int first, int update_r, const int* flags, hipStream_t st, const double* part,
                      int nblk, double omega) {
  MrArgs<T> a{x, r_out, r_in, p, alpha, n, first, update_r, flags, nrhs, part, nblk, omega};
  dispatch(mr_update_kernel<T>, a, dim3(nblocks(n, 1L << 20), (unsigned)nrhs), dim3(256), st);
}
template void launch_mr_update<double>(double2*, double2*, const double2*, const double2*, const double*, long, int, int,
                                       int, const int*, hipStream_t, const double*, int, double);
template void launch_mr_update<float>(float2*, float2*, const float2*, const float2*, const double*, long, int, int,
                                      int, const int*, hipStream_t, const double*, int, double);

template <typename T>
void launch_norm2(const cplx<T>* v, long n, int nrhs, RedArgs red, hipStream_t st) {
  NormArgs<T> a{v, n, red, nrhs};
  dispatch(norm2_kernel<T>, a, dim3(red_blocks(n), (unsigned)nrhs), dim3(256), st);
}
template void launch_norm2<double>(const double2*, long, int, RedArgs, hipStream_t);
template void launch_norm2<float>(const float2*, long, int, RedArgs, hipStream_t);

template <typename T>
static GcrArgs<T> gcr_args(long n, int nrhs, RedArgs red) {
  GcrArgs<T> a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.nrhs = nrhs;
  a.red = red;
  return a;
}

template <typename T>
void launch_gcr_mdot(const cplx<T>* Wb, long dstride, const cplx<T>* w, int k, long n, int nrhs, RedArgs red,
                     int beta_slot, int ww_slot, hipStream_t st) {
  if (k <= 0) return;
  GcrArgs<T> a = gcr_args<T>(n, nrhs, red);
  a.Wb = const_cast<cplx<T>*>(Wb); a.dstride = dstride; a.w = const_cast<cplx<T>*>(w); a.k = k;
  a.beta_slot = beta_slot; a.ww_slot = ww_slot;
  dim3 grid(red_blocks(n), (unsigned)nrhs);
  if (k <= 2) dispatch(gcr_mdot_kernel<T, 2>, a, grid, dim3(256), st);
  else if (k <= 4) dispatch(gcr_mdot_kernel<T, 4>, a, grid, dim3(256), st);
  else if (k <= 8) dispatch(gcr_mdot_kernel<T, 8>, a, grid, dim3(256), st);
  else if (k <= 16) dispatch(gcr_mdot_kernel<T, 16>, a, grid, dim3(256), st);
  else dispatch(gcr_mdot_kernel<T, 32>, a, grid, dim3(256), st);
}
template void launch_gcr_mdot<double>(const double2*, long, const double2*, int, long, int, RedArgs, int, int, hipStream_t);
template void launch_gcr_mdot<float>(const float2*, long, const float2*, int, long, int, RedArgs, int, int, hipStream_t);

template <typename T>
void launch_gcr_maxpy(cplx<T>* w, cplx<T>* z, const cplx<T>* Wb, const cplx<T>* Zb, long dstride, const cplx<T>* r, int k,
                      long n, int nrhs, RedArgs red, int beta_slot, int ww_slot, int alpha_slot, hipStream_t st) {
  GcrArgs<T> a = gcr_args<T>(n, nrhs, red);
  a.w = w; a.z = z; a.Wb = const_cast<cplx<T>*>(Wb); a.Zb = const_cast<cplx<T>*>(Zb); a.dstride = dstride;
  a.r = const_cast<cplx<T>*>(r); a.k = k;
  a.beta_slot = beta_slot; a.ww_slot = ww_slot; a.alpha_slot = alpha_slot;
  const dim3 grid(red_blocks(n), (unsigned)nrhs);
  if (k <= 1) dispatch(gcr_maxpy_kernel<T, 1>, a, grid, dim3(256), st);
  else if (k <= 2) dispatch(gcr_maxpy_kernel<T, 2>, a, grid, dim3(256), st);
  else if (k <= 4) dispatch(gcr_maxpy_kernel<T, 4>, a, grid, dim3(256), st);
  else if (k <= 8) dispatch(gcr_maxpy_kernel<T, 8>, a, grid, dim3(256), st);
  else if (k <= 16) dispatch(gcr_maxpy_kernel<T, 16>, a, grid, dim3(256), st);
  else dispatch(gcr_maxpy_kernel<T, 32>, a, grid, dim3(256), st);
}
template void launch_gcr_maxpy<double>(double2*, double2*, const double2*, const double2*, long, const double2*, int, long, int, RedArgs, int, int, int, hipStream_t);
template void launch_gcr_maxpy<float>(float2*, float2*, const float2*, const float2*, long, const float2*, int, long, int, RedArgs, int, int, int, hipStream_t);

template <typename T>
void launch_gcr_dots(const cplx<T>* Wb, long dstride, const cplx<T>* w, const cplx<T>* r, int k, long n, int nrhs,
                     RedArgs red, int beta_slot, int ww_slot, int alpha_slot, int rr_slot, int bb_slot, double tol2,
                     int* set_flags, hipStream_t st) {
  GcrArgs<T> a = gcr_args<T>(n, nrhs, red);
  a.Wb = const_cast<cplx<T>*>(Wb); a.dstride = dstride; a.w = const_cast<cplx<T>*>(w);
  a.r = const_cast<cplx<T>*>(r); a.k = k;
  a.beta_slot = beta_slot; a.ww_slot = ww_slot; a.alpha_slot = alpha_slot;
  a.rr_slot = rr_slot; a.bb_slot = bb_slot; a.tol2 = tol2; a.set_flags = set_flags;
  const dim3 grid(red_blocks(n), (unsigned)nrhs);
#define AMG_DOTS(RR)                                                                    \
  if (k <= 0) dispatch(gcr_dots_kernel<T, 0, RR>, a, grid, dim3(256), st);             \
  else if (k <= 2) dispatch(gcr_dots_kernel<T, 2, RR>, a, grid, dim3(256), st);        \
  else if (k <= 4) dispatch(gcr_dots_kernel<T, 4, RR>, a, grid, dim3(256), st);        \
  else if (k <= 6) dispatch(gcr_dots_kernel<T, 6, RR>, a, grid, dim3(256), st);        \
  else if (k <= 8) dispatch(gcr_dots_kernel<T, 8, RR>, a, grid, dim3(256), st);        \
  else if (k <= 10) dispatch(gcr_dots_kernel<T, 10, RR>, a, grid, dim3(256), st);      \
  else if (k <= 12) dispatch(gcr_dots_kernel<T, 12, RR>, a, grid, dim3(256), st);      \
  else if (k <= 16) dispatch(gcr_dots_kernel<T, 16, RR>, a, grid, dim3(256), st);      \
  else dispatch(gcr_dots_kernel<T, 32, RR>, a, grid, dim3(256), st);
  if (rr_slot >= 0) {
    AMG_DOTS(true)
  } else {
    AMG_DOTS(false)
  }
#undef AMG_DOTS
}
template void launch_gcr_dots<double>(const double2*, long, const double2*, const double2*, int, long, int, RedArgs,
                                      int, int, int, int, int, double, int*, hipStream_t);
template void launch_gcr_dots<float>(const float2*, long, const float2*, const float2*, int, long, int, RedArgs, int,
                                     int, int, int, int, double, int*, hipStream_t);

template <typename T>
void launch_gcr_update(cplx<T>* x, cplx<T>* r, const cplx<T>* z, const cplx<T>* w, long n, int nrhs, RedArgs red,
                       int alpha_slot, int rr_slot, int bb_slot, double tol2, int* set_flags, hipStream_t st) {
  GcrArgs<T> a = gcr_args<T>(n, nrhs, red);
  a.x = x; a.r = r; a.z = const_cast<cplx<T>*>(z); a.w = const_cast<cplx<T>*>(w);
  a.alpha_slot = alpha_slot; a.rr_slot = rr_slot; a.bb_slot = bb_slot; a.tol2 = tol2; a.set_flags = set_flags;
  dispatch(gcr_update_kernel<T>, a, dim3(red_blocks(n), (unsigned)nrhs), dim3(256), st);
}
template void launch_gcr_update<double>(double2*, double2*, const double2*, const double2*, long, int, RedArgs, int, int, int, double, int*, hipStream_t);
template void launch_gcr_update<float>(float2*, float2*, const float2*, const float2*, long, int, RedArgs, int, int, int, double, int*, hipStream_t);

template <typename T>
void launch_gcr_update2(cplx<T>* x, cplx<T>* r, const cplx<T>* zsrc, cplx<T>* Wb, cplx<T>* Zb, long dstride, int k,
                        long n, int nrhs, RedArgs red, int beta_slot, int alpha_slot, int rr_slot, int bb_slot,
                        double tol2, int* set_flags, hipStream_t st) {
  GcrArgs<T> a = gcr_args<T>(n, nrhs, red);
  a.x = x; a.r = r; a.zsrc = zsrc; a.Wb = Wb; a.Zb = Zb; a.dstride = dstride; a.k = k;
  a.beta_slot = beta_slot; a.alpha_slot = alpha_slot; a.rr_slot = rr_slot; a.bb_slot = bb_slot; a.tol2 = tol2;
  a.set_flags = set_flags;
  const dim3 grid(red_blocks(n), (unsigned)nrhs);
#define AMG_UPD2(RED)                                                                   \
  if (k <= 0) dispatch(gcr_update2_kernel<T, 0, RED>, a, grid, dim3(256), st);         \
  else if (k <= 2) dispatch(gcr_update2_kernel<T, 2, RED>, a, grid, dim3(256), st);    \
  else if (k <= 4) dispatch(gcr_update2_kernel<T, 4, RED>, a, grid, dim3(256), st);    \
  else if (k <= 6) dispatch(gcr_update2_kernel<T, 6, RED>, a, grid, dim3(256), st);    \
  else if (k <= 8) dispatch(gcr_update2_kernel<T, 8, RED>, a, grid, dim3(256), st);    \
  else if (k <= 10) dispatch(gcr_update2_kernel<T, 10, RED>, a, grid, dim3(256), st);  \
  else if (k <= 12) dispatch(gcr_update2_kernel<T, 12, RED>, a, grid, dim3(256), st);  \
  else if (k <= 16) dispatch(gcr_update2_kernel<T, 16, RED>, a, grid, dim3(256), st);  \
  else dispatch(gcr_update2_kernel<T, 32, RED>, a, grid, dim3(256), st);
  if (rr_slot >= 0) {
    AMG_UPD2(true)
  } else {
    AMG_UPD2(false)
  }
#undef AMG_UPD2
}
template void launch_gcr_update2<double>(double2*, double2*, const double2*, double2*, double2*, long, int, long, int,
                                         RedArgs, int, int, int, int, double, int*, hipStream_t);
template void launch_gcr_update2<float>(float2*, float2*, const float2*, float2*, float2*, long, int, long, int,
                                        RedArgs, int, int, int, int, double, int*, hipStream_t);

void launch_set_flags(int* flags, const int* inherit, const double* scal, int rr_slot, int bb_slot, double tol2,
                      int nrhs, hipStream_t st) {
  FlagArgs a{flags, inherit, scal, rr_slot, bb_slot, tol2, nrhs};
  dispatch(set_flags_kernel, a, dim3(1), dim3(64), st);
}

void launch_gather(double* out, const double* scal, int slot, int nrhs, hipStream_t st) {
  GatherArgs a{out, scal, slot, nrhs};
  dispatch(gather_kernel, a, dim3(1), dim3(64), st);
}

void launch_cg_update(double2* x, double2* r, const double2* p, const double2* q, long n, int nrhs, RedArgs red,
                      int gamma_slot, int qq_slot, int rr_slot, hipStream_t st) {
  dim3 grid(red_blocks(n), (unsigned)nrhs);
  hipLaunchKernelGGL(cg_update_kernel, grid, dim3(256), 0, st, x, r, p, q, n, red, gamma_slot, qq_slot, rr_slot);
}

void launch_cg_pupdate(double2* p, const double2* s, long n, int nrhs, const double* scal, int gnew_slot, int gold_slot,
                       hipStream_t st) {
  dim3 grid(nblocks(n, 1L << 20), (unsigned)nrhs);
  hipLaunchKernelGGL(cg_pupdate_kernel, grid, dim3(256), 0, st, p, s, n, scal, gnew_slot, gold_slot);
}

}  // namespace amg

namespace amg {
namespace {
template <typename T>
__global__ void axpy_kernel(cplx<T>* __restrict__ y, const cplx<T>* __restrict__ x, T are, T aim, long n) {
  const long ro = (long)blockIdx.y * n;
  const cplx<T> a = mk<T>(are, aim);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[ro + i] = cadd<T>(y[ro + i], cmul<T>(a, x[ro + i]));
}
template <typename T>
__global__ void scale_inv_norm_kernel(cplx<T>* __restrict__ v, const double* __restrict__ nn, long n) {
  const int rhs = blockIdx.y;
  const long ro = (long)rhs * n;
  const double q = nn[rhs];
  const T s = q > 0.0 ? (T)(1.0 / sqrt(q)) : (T)0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v[ro + i] = cscale<T>(s, v[ro + i]);
}
}  // namespace

template <typename T>
void launch_axpy(cplx<T>* y, const cplx<T>* x, double are, double aim, long n, int nrhs, hipStream_t st) {
  long nb = (n + 255) / 256; if (nb > (1L << 20)) nb = 1L << 20; if (nb < 1) nb = 1;
  hipLaunchKernelGGL((axpy_kernel<T>), dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, st, y, x, (T)are, (T)aim, n);
}
template void launch_axpy<double>(double2*, const double2*, double, double, long, int, hipStream_t);
template void launch_axpy<float>(float2*, const float2*, double, double, long, int, hipStream_t);

template <typename T>
void launch_scale_inv_norm(cplx<T>* v, const double* nn, long n, int nrhs, hipStream_t st) {
  long nb = (n + 255) / 256; if (nb > (1L << 20)) nb = 1L << 20; if (nb < 1) nb = 1;
  hipLaunchKernelGGL((scale_inv_norm_kernel<T>), dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, st, v, nn, n);
}
template void launch_scale_inv_norm<double>(double2*, const double*, long, int, hipStream_t);
template void launch_scale_inv_norm<float>(float2*, const double*, long, int, hipStream_t);
}  // namespace amg

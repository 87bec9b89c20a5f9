// Vector kernels of the smoother and the Krylov solvers: MR updates, GCR
// orthogonalisation / updates, CG on the normal equations, norms, and the
// precision / layout conversions.  All coefficients stay on the device
// (written by the last block of the producing reduction, read by the
// consumers), so a solver step needs no host round trip.
#include "common.h"
#include "kernels.h"

namespace amg {
namespace {

inline unsigned nblocks(long n, long cap) {
  long b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define GRID_STRIDE(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

template <typename Tin, typename Tout>
__global__ void convert_kernel(cplx<Tout>* __restrict__ out, const cplx<Tin>* __restrict__ in, Layout li, Layout lo) {
  const int rhs = blockIdx.y;
  const long n = li.per_rhs();
  const long ro = (long)rhs * n;
  GRID_STRIDE(i, n) {
    const int c = (int)(i / li.V);
    const long s = i - (long)c * li.V;
    const cplx<Tin> z = in[ro + li.off(s, c)];
    out[ro + lo.off(s, c)] = mk<Tout>((Tout)z.x, (Tout)z.y);
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
__global__ void mr_update_kernel(cplx<T>* __restrict__ x, cplx<T>* __restrict__ r_out, const cplx<T>* __restrict__ r_in,
                                 const cplx<T>* __restrict__ p, const double* __restrict__ alpha, long n, int first,
                                 int update_r, const int* flags) {
  const int rhs = blockIdx.y;
  if (skip_rhs(flags, rhs)) return;
  const cplx<T> a = mk<T>((T)alpha[2 * rhs], (T)alpha[2 * rhs + 1]);
  const long ro = (long)rhs * n;
  GRID_STRIDE(i, n) {
    const cplx<T> r = r_in[ro + i];
    const cplx<T> ar = cmul<T>(a, r);
    x[ro + i] = first ? ar : cadd<T>(x[ro + i], ar);
    if (update_r) r_out[ro + i] = csub<T>(r, cmul<T>(a, p[ro + i]));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void norm2_kernel(const cplx<T>* __restrict__ v, long n, RedArgs red) {
  const int rhs = blockIdx.y;
  if (skip_rhs(red.flags, rhs)) return;
  const long ro = (long)rhs * n;
  double acc[1] = {0.0};
  GRID_STRIDE(i, n) { const cplx<T> z = v[ro + i]; acc[0] += (double)z.x * z.x + (double)z.y * z.y; }
  double tot[1];
  if (grid_reduce<1>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) red.scal[red.slot + rhs] = tot[0];
}

// beta_j = <W_j, w> / <W_j, W_j>, j < k  (classical Gram-Schmidt coefficients)
template <typename T, int KM>
__global__ __launch_bounds__(256) void gcr_mdot_kernel(const cplx<T>* __restrict__ Wb, long dstride,
                                                       const cplx<T>* __restrict__ w, int k, long n, RedArgs red,
                                                       int beta_slot, int ww_slot) {
  const int rhs = blockIdx.y;
  if (skip_rhs(red.flags, rhs)) return;
  const long ro = (long)rhs * n;
  double acc[2 * KM];
#pragma unroll
  for (int j = 0; j < 2 * KM; ++j) acc[j] = 0.0;
  GRID_STRIDE(i, n) {
    const cplx<T> wi = w[ro + i];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        const cplx<T> q = Wb[(long)j * dstride + ro + i];
        acc[2 * j] += (double)q.x * wi.x + (double)q.y * wi.y;
        acc[2 * j + 1] += (double)q.x * wi.y - (double)q.y * wi.x;
      }
    }
  }
  double tot[2 * KM];
  if (grid_reduce<2 * KM>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) {
    for (int j = 0; j < k; ++j) {
      const double ww = red.scal[ww_slot + rhs * GCR_KMAX + j];
      const double s = ww > 0.0 ? 1.0 / ww : 0.0;
      red.scal[beta_slot + (rhs * GCR_KMAX + j) * 2] = tot[2 * j] * s;
      red.scal[beta_slot + (rhs * GCR_KMAX + j) * 2 + 1] = tot[2 * j + 1] * s;
    }
  }
}

// w -= sum_j beta_j W_j ; z -= sum_j beta_j Z_j ; then <w,w> and alpha = <w,r>/<w,w>
template <typename T>
__global__ __launch_bounds__(256) void gcr_maxpy_kernel(cplx<T>* __restrict__ w, cplx<T>* __restrict__ z,
                                                        const cplx<T>* __restrict__ Wb, const cplx<T>* __restrict__ Zb,
                                                        long dstride, const cplx<T>* __restrict__ r, int k, long n,
                                                        RedArgs red, int beta_slot, int ww_slot, int alpha_slot) {
  const int rhs = blockIdx.y;
  if (skip_rhs(red.flags, rhs)) return;
  const long ro = (long)rhs * n;
  const double* beta = red.scal + beta_slot + (long)rhs * GCR_KMAX * 2;
  double acc[3] = {0.0, 0.0, 0.0};
  GRID_STRIDE(i, n) {
    cplx<T> wi = w[ro + i];
    cplx<T> zi = z[ro + i];
    for (int j = 0; j < k; ++j) {
      const cplx<T> b = mk<T>((T)beta[2 * j], (T)beta[2 * j + 1]);
      wi = csub<T>(wi, cmul<T>(b, Wb[(long)j * dstride + ro + i]));
      zi = csub<T>(zi, cmul<T>(b, Zb[(long)j * dstride + ro + i]));
    }
    if (k > 0) { w[ro + i] = wi; z[ro + i] = zi; }
    const cplx<T> ri = r[ro + i];
    acc[0] += (double)wi.x * wi.x + (double)wi.y * wi.y;
    acc[1] += (double)wi.x * ri.x + (double)wi.y * ri.y;
    acc[2] += (double)wi.x * ri.y - (double)wi.y * ri.x;
  }
  double tot[3];
  if (grid_reduce<3>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) {
    const double ww = tot[0];
    red.scal[ww_slot + rhs * GCR_KMAX + k] = ww;
    const double s = ww > 0.0 ? 1.0 / ww : 0.0;
    red.scal[alpha_slot + 2 * rhs] = tot[1] * s;
    red.scal[alpha_slot + 2 * rhs + 1] = tot[2] * s;
  }
}

// x += alpha z ; r -= alpha w ; rr = <r,r> ; optionally flag rr <= tol2 * bb
template <typename T>
__global__ __launch_bounds__(256) void gcr_update_kernel(cplx<T>* __restrict__ x, cplx<T>* __restrict__ r,
                                                         const cplx<T>* __restrict__ z, const cplx<T>* __restrict__ w,
                                                         long n, RedArgs red, int alpha_slot, int rr_slot, int bb_slot,
                                                         double tol2, int* set_flags) {
  const int rhs = blockIdx.y;
  if (skip_rhs(red.flags, rhs)) return;
  const long ro = (long)rhs * n;
  const cplx<T> a = mk<T>((T)red.scal[alpha_slot + 2 * rhs], (T)red.scal[alpha_slot + 2 * rhs + 1]);
  double acc[1] = {0.0};
  GRID_STRIDE(i, n) {
    x[ro + i] = cadd<T>(x[ro + i], cmul<T>(a, z[ro + i]));
    const cplx<T> ri = csub<T>(r[ro + i], cmul<T>(a, w[ro + i]));
    r[ro + i] = ri;
    acc[0] += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  double tot[1];
  if (grid_reduce<1>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) {
    red.scal[rr_slot + rhs] = tot[0];
    if (set_flags) set_flags[rhs] = (tot[0] <= tol2 * red.scal[bb_slot + rhs]) ? 1 : 0;
  }
}

// GCR step, part 2: w' = w - sum_j beta_j W_j, z' = zsrc - sum_j beta_j Z_j
// (stored as direction k), x += alpha z', r -= alpha w', <r, r> and flags.
template <typename T>
__global__ __launch_bounds__(256) void gcr_update2_kernel(cplx<T>* __restrict__ x, cplx<T>* __restrict__ r,
                                                          const cplx<T>* zsrc, cplx<T>* Wb, cplx<T>* Zb, long dstride,
                                                          int k, long n, RedArgs red, int beta_slot, int alpha_slot,
                                                          int rr_slot, int bb_slot, double tol2, int* set_flags) {
  const int rhs = blockIdx.y;
  if (skip_rhs(red.flags, rhs)) return;
  const long ro = (long)rhs * n;
  const double* beta = red.scal + beta_slot + (long)rhs * GCR_KMAX * 2;
  const cplx<T> al = mk<T>((T)red.scal[alpha_slot + 2 * rhs], (T)red.scal[alpha_slot + 2 * rhs + 1]);
  cplx<T>* Wk = Wb + (long)k * dstride + ro;
  cplx<T>* Zk = Zb + (long)k * dstride + ro;
  double acc[1] = {0.0};
  GRID_STRIDE(i, n) {
    cplx<T> wi = Wk[i], zi = zsrc[ro + i];
    for (int j = 0; j < k; ++j) {
      const cplx<T> b = mk<T>((T)beta[2 * j], (T)beta[2 * j + 1]);
      wi = csub<T>(wi, cmul<T>(b, Wb[(long)j * dstride + ro + i]));
      zi = csub<T>(zi, cmul<T>(b, Zb[(long)j * dstride + ro + i]));
    }
    Wk[i] = wi;
    Zk[i] = zi;
    x[ro + i] = cadd<T>(x[ro + i], cmul<T>(al, zi));
    const cplx<T> ri = csub<T>(r[ro + i], cmul<T>(al, wi));
    r[ro + i] = ri;
    acc[0] += (double)ri.x * ri.x + (double)ri.y * ri.y;
  }
  double tot[1];
  if (grid_reduce<1>(acc, red.part, red.ticket, rhs, tot) && threadIdx.x == 0) {
    red.scal[rr_slot + rhs] = tot[0];
    if (set_flags) set_flags[rhs] = (tot[0] <= tol2 * red.scal[bb_slot + rhs]) ? 1 : 0;
  }
}

__global__ void set_flags_kernel(int* flags, const double* scal, int rr_slot, int bb_slot, double tol2, int nrhs) {
  const int rhs = threadIdx.x;
  if (rhs < nrhs) flags[rhs] = (scal[rr_slot + rhs] <= tol2 * scal[bb_slot + rhs]) ? 1 : 0;
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
  Layout li{V, dof, Win}, lo{V, dof, Wout};
  dim3 grid(nblocks(V * dof, 1L << 20), (unsigned)nrhs);
  hipLaunchKernelGGL((convert_kernel<Tin, Tout>), grid, dim3(256), 0, st, out, in, li, lo);
}
template void launch_convert<double, double>(double2*, const double2*, long, int, int, int, int, hipStream_t);
template void launch_convert<double, float>(float2*, const double2*, long, int, int, int, int, hipStream_t);
template void launch_convert<float, double>(double2*, const float2*, long, int, int, int, int, hipStream_t);
template void launch_convert<float, float>(float2*, const float2*, long, int, int, int, int, hipStream_t);

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
                      int nrhs, int first, int update_r, const int* flags, hipStream_t st) {
  dim3 grid(nblocks(n, 1L << 20), (unsigned)nrhs);
  hipLaunchKernelGGL((mr_update_kernel<T>), grid, dim3(256), 0, st, x, r_out, r_in, p, alpha, n, first, update_r, flags);
}
template void launch_mr_update<double>(double2*, double2*, const double2*, const double2*, const double*, long, int, int, int, const int*, hipStream_t);
template void launch_mr_update<float>(float2*, float2*, const float2*, const float2*, const double*, long, int, int, int, const int*, hipStream_t);

template <typename T>
void launch_norm2(const cplx<T>* v, long n, int nrhs, RedArgs red, hipStream_t st) {
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
  hipLaunchKernelGGL((norm2_kernel<T>), grid, dim3(256), 0, st, v, n, red);
}
template void launch_norm2<double>(const double2*, long, int, RedArgs, hipStream_t);
template void launch_norm2<float>(const float2*, long, int, RedArgs, hipStream_t);

template <typename T>
void launch_gcr_mdot(const cplx<T>* Wb, long dstride, const cplx<T>* w, int k, long n, int nrhs, RedArgs red,
                     int beta_slot, int ww_slot, hipStream_t st) {
  if (k <= 0) return;
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
  if (k <= 4)
    hipLaunchKernelGGL((gcr_mdot_kernel<T, 4>), grid, dim3(256), 0, st, Wb, dstride, w, k, n, red, beta_slot, ww_slot);
  else if (k <= 8)
    hipLaunchKernelGGL((gcr_mdot_kernel<T, 8>), grid, dim3(256), 0, st, Wb, dstride, w, k, n, red, beta_slot, ww_slot);
  else if (k <= 16)
    hipLaunchKernelGGL((gcr_mdot_kernel<T, 16>), grid, dim3(256), 0, st, Wb, dstride, w, k, n, red, beta_slot, ww_slot);
  else
    hipLaunchKernelGGL((gcr_mdot_kernel<T, 32>), grid, dim3(256), 0, st, Wb, dstride, w, k, n, red, beta_slot, ww_slot);
}
template void launch_gcr_mdot<double>(const double2*, long, const double2*, int, long, int, RedArgs, int, int, hipStream_t);
template void launch_gcr_mdot<float>(const float2*, long, const float2*, int, long, int, RedArgs, int, int, hipStream_t);

template <typename T>
void launch_gcr_maxpy(cplx<T>* w, cplx<T>* z, const cplx<T>* Wb, const cplx<T>* Zb, long dstride, const cplx<T>* r, int k,
                      long n, int nrhs, RedArgs red, int beta_slot, int ww_slot, int alpha_slot, hipStream_t st) {
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
  hipLaunchKernelGGL((gcr_maxpy_kernel<T>), grid, dim3(256), 0, st, w, z, Wb, Zb, dstride, r, k, n, red, beta_slot,
                     ww_slot, alpha_slot);
}
template void launch_gcr_maxpy<double>(double2*, double2*, const double2*, const double2*, long, const double2*, int, long, int, RedArgs, int, int, int, hipStream_t);
template void launch_gcr_maxpy<float>(float2*, float2*, const float2*, const float2*, long, const float2*, int, long, int, RedArgs, int, int, int, hipStream_t);

template <typename T>
void launch_gcr_update(cplx<T>* x, cplx<T>* r, const cplx<T>* z, const cplx<T>* w, long n, int nrhs, RedArgs red,
                       int alpha_slot, int rr_slot, int bb_slot, double tol2, int* set_flags, hipStream_t st) {
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
  hipLaunchKernelGGL((gcr_update_kernel<T>), grid, dim3(256), 0, st, x, r, z, w, n, red, alpha_slot, rr_slot, bb_slot,
                     tol2, set_flags);
}
template void launch_gcr_update<double>(double2*, double2*, const double2*, const double2*, long, int, RedArgs, int, int, int, double, int*, hipStream_t);
template void launch_gcr_update<float>(float2*, float2*, const float2*, const float2*, long, int, RedArgs, int, int, int, double, int*, hipStream_t);

template <typename T>
void launch_gcr_update2(cplx<T>* x, cplx<T>* r, const cplx<T>* zsrc, cplx<T>* Wb, cplx<T>* Zb, long dstride, int k,
                        long n, int nrhs, RedArgs red, int beta_slot, int alpha_slot, int rr_slot, int bb_slot,
                        double tol2, int* set_flags, hipStream_t st) {
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
  hipLaunchKernelGGL((gcr_update2_kernel<T>), grid, dim3(256), 0, st, x, r, zsrc, Wb, Zb, dstride, k, n, red,
                     beta_slot, alpha_slot, rr_slot, bb_slot, tol2, set_flags);
}
template void launch_gcr_update2<double>(double2*, double2*, const double2*, double2*, double2*, long, int, long, int,
                                         RedArgs, int, int, int, int, double, int*, hipStream_t);
template void launch_gcr_update2<float>(float2*, float2*, const float2*, float2*, float2*, long, int, long, int,
                                        RedArgs, int, int, int, int, double, int*, hipStream_t);

template <typename T>
void launch_set_flags(int* flags, const double* scal, int rr_slot, int bb_slot, double tol2, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(set_flags_kernel, dim3(1), dim3(64), 0, st, flags, scal, rr_slot, bb_slot, tol2, nrhs);
}
template void launch_set_flags<double>(int*, const double*, int, int, double, int, hipStream_t);
template void launch_set_flags<float>(int*, const double*, int, int, double, int, hipStream_t);

void launch_cg_update(double2* x, double2* r, const double2* p, const double2* q, long n, int nrhs, RedArgs red,
                      int gamma_slot, int qq_slot, int rr_slot, hipStream_t st) {
  dim3 grid(nblocks(n, RED_MAX_BLOCKS), (unsigned)nrhs);
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

// Exact solve of the coarsest level.  The paper solves its coarsest lattice
// exactly (the V-cycle's recursion ends in a direct solve); for a coarsest
// level of at most a few thousand unknowns this library forms the dense
// matrix of the Galerkin operator, inverts it once per setup (or mass
// change) by Gauss-Jordan elimination with partial pivoting in FP64, and
// then every coarsest solve is one dense matrix-vector product.
//
// Elimination: in-place Gauss-Jordan without row exchanges.  Step k picks
// the unused row p with the largest |re| + |im| in column k, scales row p by
// 1/a (a = A[p][k]) and eliminates column k from every other row; the column
// of the inverse that this step produces is stored in place of column k.
// After N steps the inverse is the stored matrix with rows taken in pivot
// order and columns in inverse pivot order:
//   Ainv[k][j] = A_final[piv[k]][pinv[j]],  pinv[piv[m]] = m.
// One launch per step reads the previous matrix and writes the next one
// (two buffers), so no block reads a value another block of the same launch
// writes; the pivot of step k + 1 is found by the blocks that produce
// column k + 1 (a 64-bit atomic maximum of (magnitude bits, ~row)).
#include <utility>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace amg {
namespace {

__device__ __forceinline__ void dcoords(long site, const int (&dims)[4], int nd, int (&x)[4]) {
  long rem = site;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    x[mu] = 0;
    if (mu < nd) { x[mu] = (int)(rem % dims[mu]); rem /= dims[mu]; }
  }
}

__device__ __forceinline__ long dneighbour(long site, const int (&x)[4], const int (&dims)[4], int dir) {
  const int mu = dir >> 1;
  long stride = 1;
#pragma unroll
  for (int nu = 0; nu < 3; ++nu)
    if (nu < mu) stride *= dims[nu];
  const int L = at4(dims, mu);
  const int xm = at4(x, mu);
  if ((dir & 1) == 0) return (xm == L - 1) ? site - (long)(L - 1) * stride : site + stride;
  return (xm == 0) ? site + (long)(L - 1) * stride : site - stride;
}

// Row i = site * nc + row of the dense operator (zeroed beforehand): every
// block Y[site][k] adds its row into the columns of the neighbour it couples
// to (coarse extents 1 or 2 make neighbours coincide, hence +=).  One thread
// owns one row, so the sums need no atomics.
__global__ __launch_bounds__(256) void dense_assemble_kernel(double2* __restrict__ A, const double2* __restrict__ Y,
                                                             CoarseGeom g, long N) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int nc = g.nc;
  const int ndir = 2 * g.nd + 1;
  const long site = i / nc;
  const int row = (int)(i - site * nc);
  int x[4];
  dcoords(site, g.dims, g.nd, x);
  gptr<double2> Arow = gl(A) + i * N;
  gptr<const double2> Yg = gl(Y);
  for (int k = 0; k < ndir; ++k) {
    const long nb = (k == 0) ? site : dneighbour(site, x, g.dims, k - 1);
    gptr<const double2> Yk = Yg + ((site * ndir + k) * nc) * (long)nc + row;
    for (int col = 0; col < nc; ++col) {
      const double2 y = Yk[(long)col * nc];
      double2 v = Arow[nb * nc + col];
      v.x += y.x;
      v.y += y.y;
      Arow[nb * nc + col] = v;
    }
  }
}

// pivot key: magnitude bits high, ~row low (larger magnitude wins, then the smaller row)
__device__ __forceinline__ unsigned long long pivot_key(double2 v, long i) {
  const float m = (float)(fabs(v.x) + fabs(v.y));
  return ((unsigned long long)__float_as_uint(m) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
}

constexpr int GJ_T = 64;      // tile: 64 rows x 64 columns per block of 256 threads
constexpr int GJ_ROWS = GJ_T / 4;

// pivot of column 0: every row is a candidate
__global__ __launch_bounds__(256) void gj_first_pivot_kernel(const double2* __restrict__ A, long N,
                                                             unsigned long long* __restrict__ key) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long kk = 0;
  if (i < N) kk = pivot_key(gl(A)[i * N], i);
  __shared__ unsigned long long sh[256];
  sh[threadIdx.x] = kk;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && sh[threadIdx.x + s] > sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0] != 0) atomicMax(key, sh[0]);
}

__global__ __launch_bounds__(256) void gj_step_kernel(const double2* __restrict__ Ain, double2* __restrict__ Aout,
                                                      long N, long k, unsigned long long* __restrict__ key,
                                                      int* __restrict__ piv, int* __restrict__ used,
                                                      int* __restrict__ err) {
  const unsigned long long kk = __hip_atomic_load(key + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const long p = (long)(0xFFFFFFFFu - (unsigned)(kk & 0xFFFFFFFFull));
  const bool singular = (kk >> 32) == 0 || p >= N;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    if (singular) {
      gl(err)[0] = 1;
    } else {
      gl(piv)[k] = (int)p;
      gl(used)[p] = 1;
    }
  }
  if (singular) return;  // uniform: the host reports the error after the sweep
  gptr<const double2> A = gl(Ain);
  const double2 a = A[p * N + k];
  const double na = a.x * a.x + a.y * a.y;
  const double2 inv = make_double2(a.x / na, -a.y / na);
  const long r0 = (long)blockIdx.y * GJ_T, c0 = (long)blockIdx.x * GJ_T;
  __shared__ double2 colk[GJ_T], rowp[GJ_T];
  const int t = threadIdx.x;
  if (t < GJ_T) {
    double2 v = make_double2(0.0, 0.0);
    if (r0 + t < N) v = A[(r0 + t) * N + k];
    colk[t] = v;
  } else if (t < 2 * GJ_T) {
    double2 v = make_double2(0.0, 0.0);
    if (c0 + t - GJ_T < N) v = A[p * N + c0 + t - GJ_T];
    rowp[t - GJ_T] = v;
  }
  __syncthreads();
  const int lane = t & 63, wave = t >> 6;
  const long c = c0 + lane;
  const double2 rp = cmul<double>(rowp[lane], inv);  // scaled pivot row entry
  const bool next_col = (c == k + 1);
  unsigned long long best = 0;
  if (c < N) {
    gptr<double2> Out = gl(Aout);
    for (int q = 0; q < GJ_ROWS; ++q) {
      const long i = r0 + wave + 4 * q;
      if (i >= N) break;
      double2 o;
      if (i == p) {
        o = (c == k) ? inv : rp;
      } else {
        const double2 f = colk[i - r0];
        if (c == k) {
          const double2 fi = cmul<double>(f, inv);
          o = make_double2(-fi.x, -fi.y);
        } else {
          const double2 v = A[i * N + c];
          o = make_double2(v.x - (f.x * rp.x - f.y * rp.y), v.y - (f.x * rp.y + f.y * rp.x));
        }
      }
      Out[i * N + c] = o;
      if (next_col && i != p && !gl(used)[i]) {
        const unsigned long long kq = pivot_key(o, i);
        best = kq > best ? kq : best;
      }
    }
  }
  // pivot candidates of column k + 1: one lane per wave holds them
  if (k + 1 < N && c0 <= k + 1 && k + 1 < c0 + GJ_T) {
    __shared__ unsigned long long wb[4];
    if (next_col) wb[wave] = best;
    __syncthreads();
    if (t == 0) {
      unsigned long long m = wb[0];
      for (int w = 1; w < 4; ++w) m = wb[w] > m ? wb[w] : m;
      if (m != 0) atomicMax(key + k + 1, m);
    }
  }
}

// (after a singular sweep the pivot records are incomplete: indices outside
// [0, N) are skipped here and give NaN in the gather; the host reports the error)
__global__ void gj_invperm_kernel(const int* __restrict__ piv, int* __restrict__ pinv, long N) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const int p = gl(piv)[m];
  if (p >= 0 && p < N) gl(pinv)[p] = (int)m;
}

__global__ __launch_bounds__(256) void gj_gather_kernel(const double2* __restrict__ Af, const int* __restrict__ piv,
                                                        const int* __restrict__ pinv, double2* __restrict__ Ainv,
                                                        float2* __restrict__ Ainv32, long N) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * N) return;
  const long k = idx / N, j = idx - k * N;
  const int pk = gl(piv)[k], pj = gl(pinv)[j];
  double2 v = make_double2(__builtin_nan(""), __builtin_nan(""));
  if (pk >= 0 && pk < N && pj >= 0 && pj < N) v = gl(Af)[(long)pk * N + pj];
  gl(Ainv)[idx] = v;
  if (Ainv32) gl(Ainv32)[idx] = make_float2((float)v.x, (float)v.y);
}

// x[rhs] = Ainv b[rhs]: one wave per row, lanes stride along the row
// (coalesced), R right-hand sides per pass so the row is read once for them.
template <typename T>
struct DenseArgs {
  cplx<T>* x;
  const cplx<T>* b;
  const cplx<T>* Ainv;
  long N;
  int nrhs;
  const int* flags;
};

template <typename T, int R>
__global__ __launch_bounds__(256) void dense_apply_kernel(DenseArgs<T> a0, const DenseArgs<T>* batch) {
  AMG_PICK(a, DenseArgs<T>)
  const int rb = blockIdx.y * R;
  if (rb >= a.nrhs) return;
  const int lane = threadIdx.x & 63;
  const long i = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.N) return;
  gptr<const cplx<T>> row = gl(a.Ainv) + i * a.N;
  gptr<const cplx<T>> b = gl(a.b);
  double accr[R], acci[R];
#pragma unroll
  for (int r = 0; r < R; ++r) accr[r] = acci[r] = 0.0;
  for (long j = lane; j < a.N; j += 64) {
    const cplx<T> m = row[j];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (rb + r >= a.nrhs) break;
      const cplx<T> v = b[(long)(rb + r) * a.N + j];
      accr[r] += (double)m.x * v.x - (double)m.y * v.y;
      acci[r] += (double)m.x * v.y + (double)m.y * v.x;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (rb + r >= a.nrhs) break;
    const double sr = wave_sum(accr[r]);
    const double si = wave_sum(acci[r]);
    if (lane == 0 && !skip_rhs(a.flags, rb + r)) gl(a.x)[(long)(rb + r) * a.N + i] = mk<T>((T)sr, (T)si);
  }
}

}  // namespace

void launch_dense_assemble(double2* A, const double2* Y, const CoarseGeom& g, hipStream_t st) {
  const long N = g.V * g.nc;
  launch_fill<double>(A, nullptr, N * N, 1, st);
  hipLaunchKernelGGL(dense_assemble_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, A, Y, g, N);
}

void launch_gj_invert(double2* A, double2* B, long N, unsigned long long* key, int* piv, int* used, int* pinv,
                      int* err, double2* Ainv, float2* Ainv32, hipStream_t st) {
  // key, used and err start at zero (fill kernels: this may be captured)
  launch_fill<double>(reinterpret_cast<double2*>(key), nullptr, (N + 1) / 2, 1, st);
  launch_fill<float>(reinterpret_cast<float2*>(used), nullptr, (N + 1) / 2, 1, st);
  launch_fill<float>(reinterpret_cast<float2*>(err), nullptr, 1, 1, st);
  hipLaunchKernelGGL(gj_first_pivot_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, A, N, key);
  const unsigned nt = (unsigned)((N + GJ_T - 1) / GJ_T);
  double2* src = A;
  double2* dst = B;
  for (long k = 0; k < N; ++k) {
    hipLaunchKernelGGL(gj_step_kernel, dim3(nt, nt), dim3(256), 0, st, src, dst, N, k, key, piv, used, err);
    std::swap(src, dst);
  }
  hipLaunchKernelGGL(gj_invperm_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, piv, pinv, N);
  hipLaunchKernelGGL(gj_gather_kernel, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, st, src, piv, pinv, Ainv,
                     Ainv32, N);
}

template <typename T>
void launch_dense_apply(cplx<T>* x, const cplx<T>* b, const cplx<T>* Ainv, long N, int nrhs, const int* flags,
                        hipStream_t st) {
  DenseArgs<T> a{x, b, Ainv, N, nrhs, flags};
  const dim3 block(256);
  const unsigned gx = (unsigned)((N + 3) / 4);
  if (nrhs >= 8) dispatch(dense_apply_kernel<T, 8>, a, dim3(gx, (nrhs + 7) / 8), block, st);
  else if (nrhs >= 4) dispatch(dense_apply_kernel<T, 4>, a, dim3(gx, (nrhs + 3) / 4), block, st);
  else if (nrhs >= 2) dispatch(dense_apply_kernel<T, 2>, a, dim3(gx, (nrhs + 1) / 2), block, st);
  else dispatch(dense_apply_kernel<T, 1>, a, dim3(gx, 1), block, st);
}

template void launch_dense_apply<double>(double2*, const double2*, const double2*, long, int, const int*,
                                         hipStream_t);
template void launch_dense_apply<float>(float2*, const float2*, const float2*, long, int, const int*, hipStream_t);

}  // namespace amg

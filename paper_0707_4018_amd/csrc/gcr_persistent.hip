// Persistent coarsest-level solve for the 2d hierarchy (N_c = 16): the whole
// restarted GCR of the coarsest level (see level_gcr in the runtime for the
// iteration it reproduces) runs in one cooperative launch.  Phases are
// separated by grid barriers; every block reduces the partial sums of all
// blocks in the same fixed order, so control decisions (convergence, restart)
// are identical in every block and deterministic.
//
// Barrier: monotonic arrival counter per right-hand side, zeroed before the
// launch.  Waiting is bounded: after ~2^24 polls, or once any block has
// recorded a timeout, a block records the timeout and proceeds, so every
// wave reaches the end of the kernel; the host turns the flag into an error.
#include "common.h"
#include "kernels.h"

namespace amg {
namespace {

constexpr int PG_THREADS = 256;
constexpr int PG_WAVES = PG_THREADS / 64;
constexpr int PG_NQ = 2 * GCR_KMAX + 3;  // partial sums per block

struct PgCtl {
  unsigned epoch;
};

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblk, PgCtl& c, int* err) {
  __syncthreads();  // the block's stores are complete before thread 0 releases them
  c.epoch += 1;
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    const unsigned target = c.epoch * nblk;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ __forceinline__ int nbr_coarse(long site, const int* x, const int* dims, int nd, int dir, long* out) {
  const int mu = dir >> 1;
  long stride = 1;
  for (int nu = 0; nu < mu; ++nu) stride *= dims[nu];
  const int L = dims[mu];
  if ((dir & 1) == 0) *out = (x[mu] == L - 1) ? site - (long)(L - 1) * stride : site + stride;
  else *out = (x[mu] == 0) ? site + (long)(L - 1) * stride : site - stride;
  return 0;
}

template <typename T>
struct PgArgs {
  const cplx<T>* Y;
  CoarseGeom g;
  const cplx<T>* b;
  cplx<T>* x;
  cplx<T>* r;
  cplx<T>* Zb;
  cplx<T>* Wb;
  long dstride;   // between stored directions (n * nrhs)
  int m, maxiter;
  double tol2;
  double* part;   // [nrhs][2][nblk][PG_NQ]
  unsigned* bar;  // [nrhs]
  int* err;
  int* iters;     // [nrhs]
};

// One wave computes (A v)(site) for the 16 rows of `site` (N_c = 16); the
// result ends in lanes lane < LPC, rows lane*R .. lane*R + R - 1.
template <typename T>
__device__ __forceinline__ void wave_apply16(const PgArgs<T>& a, const cplx<T>* __restrict__ v, long site,
                                             cplx<T> (&acc)[(sizeof(T) == 4) ? 2 : 1]) {
  constexpr int NC = 16;
  constexpr int R = (sizeof(T) == 4) ? 2 : 1;
  constexpr int LPC = NC / R;
  constexpr int CPI = 64 / LPC;
  const int lane = threadIdx.x & 63;
  const int cg = lane / LPC, rg = lane - cg * LPC;
  const int nd = a.g.nd, ndir = 2 * nd + 1;
  int xc[4];
  long rem = site;
  for (int mu = 0; mu < nd; ++mu) { xc[mu] = (int)(rem % a.g.dims[mu]); rem /= a.g.dims[mu]; }
  long nbs[9];
  nbs[0] = site;
  for (int k = 1; k < ndir; ++k) nbr_coarse(site, xc, a.g.dims, nd, k - 1, &nbs[k]);
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = mk<T>(0, 0);
  const cplx<T>* __restrict__ Ys = a.Y + site * (long)ndir * NC * NC;
  for (int gc = cg; gc < ndir * NC; gc += CPI) {
    const int k = gc / NC, col = gc - k * NC;
    const cplx<T> e = v[nbs[k] * NC + col];
    const cplx<T>* y = Ys + (long)gc * NC + rg * R;
#pragma unroll
    for (int i = 0; i < R; ++i) cfma<T>(acc[i], y[i], e);
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
#pragma unroll
    for (int o = LPC; o < 64; o <<= 1) {
      acc[i].x += __shfl_xor(acc[i].x, o, 64);
      acc[i].y += __shfl_xor(acc[i].y, o, 64);
    }
  }
}

// Block partial sums of nq values held per thread in LDS scratch, then the
// grid reduction after the barrier: every block sums all partials in order.
// Partials alternate between two buffers (publish counter parity): a block
// cannot publish twice before every block has read the first publication,
// because a grid barrier separates consecutive publications.
template <int NQMAX>
struct Reducer {
  double* sh;  // [PG_WAVES][NQMAX] in LDS
  double* part0;  // this rhs's two partial buffers, each [nblk][PG_NQ]
  long half;
  unsigned pub = 0;
  __device__ void clear(int nq) {
    for (int q = threadIdx.x; q < PG_WAVES * NQMAX; q += blockDim.x) sh[q] = 0.0;
    __syncthreads();
  }
  // add a per-lane value to the wave's slot q (wave reduction, lane 0 adds)
  __device__ void add(int q, double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[(threadIdx.x >> 6) * NQMAX + q] += v;
  }
  __device__ void publish(int blk, int nq) {
    __syncthreads();
    double* part = part0 + (pub & 1u) * half;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      double s = 0.0;
      for (int w = 0; w < PG_WAVES; ++w) s += sh[w * NQMAX + q];
      part[(long)blk * PG_NQ + q] = s;
    }
  }
  // after the barrier: totals of all blocks into tot[0..nq) (LDS), fixed order
  __device__ void total(int nblk, int nq, double* tot) {
    const double* part = part0 + (pub & 1u) * half;
    pub += 1;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      double s = 0.0;
      for (int bk = 0; bk < nblk; ++bk)
        s += __hip_atomic_load(&part[(long)bk * PG_NQ + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tot[q] = s;
    }
    __syncthreads();
  }
};

template <typename T>
__global__ __launch_bounds__(PG_THREADS) void gcr16_persistent_kernel(PgArgs<T> a) {
  constexpr int NC = 16;
  constexpr int R = (sizeof(T) == 4) ? 2 : 1;
  constexpr int LPC = NC / R;
  __shared__ double sh_red[PG_WAVES * PG_NQ];
  __shared__ double tot[PG_NQ];
  __shared__ double wwh[GCR_KMAX];
  __shared__ double coef[2 * GCR_KMAX + 2];
  const int rhs = blockIdx.y;
  const int blk = blockIdx.x;
  const unsigned nblk = gridDim.x;
  const long V = a.g.V;
  const long n = V * NC;
  const long ro = (long)rhs * n;
  const cplx<T>* __restrict__ b = a.b + ro;
  cplx<T>* __restrict__ x = a.x + ro;
  cplx<T>* __restrict__ r = a.r + ro;
  unsigned* bar = a.bar + rhs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = lane / LPC, rg = lane - cg * LPC;
  Reducer<PG_NQ> red{sh_red, a.part + (long)rhs * 2 * nblk * PG_NQ, (long)nblk * PG_NQ};
  PgCtl ctl{0};
  const long tstride = (long)nblk * PG_THREADS;
  const long t0 = (long)blk * PG_THREADS + threadIdx.x;

  // x = 0, r = b, bb = <b, b>
  red.clear(1);
  {
    double s = 0.0;
    for (long i = t0; i < n; i += tstride) {
      const cplx<T> v = b[i];
      x[i] = mk<T>(0, 0);
      r[i] = v;
      s += (double)v.x * v.x + (double)v.y * v.y;
    }
    red.add(0, s);
  }
  red.publish(blk, 1);
  grid_barrier(bar, nblk, ctl, a.err);
  red.total(nblk, 1, tot);
  const double bb = tot[0];
  bool done = (a.tol2 >= 1.0) ? true : (bb == 0.0);
  int it = 0;
  for (; it < a.maxiter && !done; ++it) {
    const int k = it % a.m;
    if (k == 0 && it > 0) {
      // restart: r = b - A x
      for (long site = (long)blk * PG_WAVES + wave; site < V; site += (long)nblk * PG_WAVES) {
        cplx<T> acc[R];
        wave_apply16<T>(a, x, site, acc);
        if (cg == 0)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const long idx = site * NC + rg * R + i;
            r[idx] = csub<T>(b[idx], acc[i]);
          }
      }
      grid_barrier(bar, nblk, ctl, a.err);
    }
    cplx<T>* __restrict__ Wk = a.Wb + (long)k * a.dstride + ro;
    cplx<T>* __restrict__ Zk = a.Zb + (long)k * a.dstride + ro;
    // phase B: w = A r, z = r, dots <W_j, w> (j < k)
    const int nq1 = 2 * k;
    red.clear(nq1 + 1);
    for (long site = (long)blk * PG_WAVES + wave; site < V; site += (long)nblk * PG_WAVES) {
      cplx<T> acc[R];
      wave_apply16<T>(a, r, site, acc);
      for (int j = 0; j < k; ++j) {
        double dr = 0.0, di = 0.0;
        if (cg == 0) {
          const cplx<T>* Wj = a.Wb + (long)j * a.dstride + ro;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const cplx<T> q = Wj[site * NC + rg * R + i];
            dr += (double)q.x * acc[i].x + (double)q.y * acc[i].y;
            di += (double)q.x * acc[i].y - (double)q.y * acc[i].x;
          }
        }
        red.add(2 * j, dr);
        red.add(2 * j + 1, di);
      }
      if (cg == 0)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const long idx = site * NC + rg * R + i;
          Wk[idx] = acc[i];
          Zk[idx] = r[idx];
        }
    }
    red.publish(blk, nq1);
    grid_barrier(bar, nblk, ctl, a.err);
    red.total(nblk, nq1, tot);
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      const double s = wwh[j] > 0.0 ? 1.0 / wwh[j] : 0.0;
      coef[2 * j] = tot[2 * j] * s;
      coef[2 * j + 1] = tot[2 * j + 1] * s;
    }
    __syncthreads();
    // phase C: w -= sum beta_j W_j, z -= sum beta_j Z_j; <w,w>, <w,r>
    red.clear(3);
    {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (long i = t0; i < n; i += tstride) {
        cplx<T> wi = Wk[i], zi = Zk[i];
        for (int j = 0; j < k; ++j) {
          const cplx<T> bj = mk<T>((T)coef[2 * j], (T)coef[2 * j + 1]);
          wi = csub<T>(wi, cmul<T>(bj, a.Wb[(long)j * a.dstride + ro + i]));
          zi = csub<T>(zi, cmul<T>(bj, a.Zb[(long)j * a.dstride + ro + i]));
        }
        if (k > 0) { Wk[i] = wi; Zk[i] = zi; }
        const cplx<T> ri = r[i];
        s0 += (double)wi.x * wi.x + (double)wi.y * wi.y;
        s1 += (double)wi.x * ri.x + (double)wi.y * ri.y;
        s2 += (double)wi.x * ri.y - (double)wi.y * ri.x;
      }
      red.add(0, s0);
      red.add(1, s1);
      red.add(2, s2);
    }
    red.publish(blk, 3);
    grid_barrier(bar, nblk, ctl, a.err);
    red.total(nblk, 3, tot);
    if (threadIdx.x == 0) {
      const double ww = tot[0];
      wwh[k] = ww;
      const double s = ww > 0.0 ? 1.0 / ww : 0.0;
      coef[2 * GCR_KMAX] = tot[1] * s;
      coef[2 * GCR_KMAX + 1] = tot[2] * s;
    }
    __syncthreads();
    // phase D: x += alpha z, r -= alpha w, rr
    red.clear(1);
    {
      const cplx<T> al = mk<T>((T)coef[2 * GCR_KMAX], (T)coef[2 * GCR_KMAX + 1]);
      double s = 0.0;
      for (long i = t0; i < n; i += tstride) {
        x[i] = cadd<T>(x[i], cmul<T>(al, Zk[i]));
        const cplx<T> ri = csub<T>(r[i], cmul<T>(al, Wk[i]));
        r[i] = ri;
        s += (double)ri.x * ri.x + (double)ri.y * ri.y;
      }
      red.add(0, s);
    }
    red.publish(blk, 1);
    grid_barrier(bar, nblk, ctl, a.err);
    red.total(nblk, 1, tot);
    done = tot[0] <= a.tol2 * bb;
  }
  if (blk == 0 && threadIdx.x == 0) a.iters[rhs] = it;
}

}  // namespace

template <typename T>
hipError_t launch_gcr16_persistent(const cplx<T>* Y, const CoarseGeom& g, const cplx<T>* b, cplx<T>* x, cplx<T>* r,
                                   cplx<T>* Zb, cplx<T>* Wb, long dstride, int m, int maxiter, double tol2, int nrhs,
                                   int nblk, double* part, unsigned* bar, int* err, int* iters, hipStream_t st,
                                   bool cooperative) {
  PgArgs<T> a{Y, g, b, x, r, Zb, Wb, dstride, m, maxiter, tol2, part, bar, err, iters};
  if (cooperative) {
    void* args[] = {&a};
    return hipLaunchCooperativeKernel((const void*)gcr16_persistent_kernel<T>, dim3((unsigned)nblk, (unsigned)nrhs),
                                      dim3(PG_THREADS), args, 0, st);
  }
  // plain launch: the grid is far below one block per compute unit, and the
  // bounded barrier wait ends the kernel with an error flag should a block
  // ever not be resident
  hipLaunchKernelGGL(gcr16_persistent_kernel<T>, dim3((unsigned)nblk, (unsigned)nrhs), dim3(PG_THREADS), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_gcr16_persistent<double>(const double2*, const CoarseGeom&, const double2*, double2*,
                                                    double2*, double2*, double2*, long, int, int, double, int, int,
                                                    double*, unsigned*, int*, int*, hipStream_t, bool);
template hipError_t launch_gcr16_persistent<float>(const float2*, const CoarseGeom&, const float2*, float2*, float2*,
                                                   float2*, float2*, long, int, int, double, int, int, double*,
                                                   unsigned*, int*, int*, hipStream_t, bool);

int gcr16_partials_per_block() { return PG_NQ; }

}  // namespace amg

// Persistent coarsest-level solve (N_c = 16): the whole restarted GCR of the
// coarsest level (the iteration level_gcr in the runtime issues as separate
// launches, reproduced step for step) runs in one cooperative launch.
// Phases are separated by grid barriers; every block reduces the partial
// sums of all blocks in the same fixed order, so control decisions
// (convergence, restart) are identical in every block and deterministic.
//
// Ownership: wave w of block b owns the sites b*4 + w + t*(4*nblk) in every
// phase, and the lanes of its first column group own their rows.  Only the
// stencil reads data of other blocks (the neighbours' entries of r, and of x
// at a restart); those two vectors are written and read with agent-scope
// atomic accesses (written through to the memory side, not served from a
// stale line of another XCD's L2), everything else is private to its owner.
// That makes the barrier cheap: every thread waits until its stores are
// complete, then the block arrives — no release fence (which on this chip
// writes back the whole L2 of the XCD).
//
// Barrier: monotonic arrival counter per right-hand side, zeroed before the
// launch.  Waiting is bounded: after ~2^24 polls, or once any block has
// recorded a timeout, a block records the timeout and proceeds, so every
// wave reaches the end of the kernel; the host turns the flag into an error.
#include <cstring>

#include "common.h"
#include "kernels.h"

namespace amg {
namespace {

constexpr int PG_THREADS = 256;
constexpr int PG_WAVES = PG_THREADS / 64;
constexpr int PG_NQ = 2 * GCR_KMAX + 3;  // partial sums per block

// agent-coherent accesses of r and x
__device__ __forceinline__ float2 ld_coh(const float2* p) {
  const unsigned long long u = __hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<float2*>(p)),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  float2 v;
  memcpy(&v, &u, sizeof(v));
  return v;
}
__device__ __forceinline__ double2 ld_coh(const double2* p) {
  double* q = reinterpret_cast<double*>(const_cast<double2*>(p));
  return make_double2(__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_coh(float2* p, float2 v) {
  unsigned long long u;
  memcpy(&u, &v, sizeof(u));
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(double2* p, double2 v) {
  double* q = reinterpret_cast<double*>(p);
  __hip_atomic_store(q, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblk, unsigned& epoch, int* err) {
  wait_stores_complete();  // this thread's stores (r, x, partial sums) are complete
  __syncthreads();
  epoch += 1;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = epoch * nblk;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 24) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
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

// (A v)(site) for the 16 rows of `site` by one wave (NDIR = 2 nd + 1 blocks
// of the stencil); v is read with agent-coherent loads.  The result ends in
// the lanes of column group 0: lane rg holds rows rg*R .. rg*R + R - 1.
template <typename T, int NDIR>
__device__ __forceinline__ void pg_apply(gptr<const cplx<T>> Y, const CoarseGeom& g, const cplx<T>* v, long site,
                                         int cg, int rg, cplx<T> (&acc)[(sizeof(T) == 4) ? 2 : 1]) {
  constexpr int NC = 16;
  constexpr int R = (sizeof(T) == 4) ? 2 : 1;
  constexpr int LPC = NC / R;
  constexpr int CPI = 64 / LPC;
  constexpr int NQ = NC / CPI;
  constexpr int ND = (NDIR - 1) / 2;
  int xc[4];
  long stride[4];
  {
    long rem = site, st = 1;
#pragma unroll
    for (int mu = 0; mu < ND; ++mu) {
      xc[mu] = (int)(rem % g.dims[mu]);
      rem /= g.dims[mu];
      stride[mu] = st;
      st *= g.dims[mu];
    }
  }
  long nbs[NDIR];
  nbs[0] = site;
#pragma unroll
  for (int mu = 0; mu < ND; ++mu) {
    const int L = g.dims[mu];
    nbs[1 + 2 * mu] = (xc[mu] == L - 1) ? site - (long)(L - 1) * stride[mu] : site + stride[mu];
    nbs[2 + 2 * mu] = (xc[mu] == 0) ? site + (long)(L - 1) * stride[mu] : site - stride[mu];
  }
  gptr<const cplx<T>> Ys = Y + site * (long)NDIR * NC * NC + rg * R;
  cplx<T> ev[NDIR][NQ], yv[NDIR][NQ][R];
#pragma unroll
  for (int k = 0; k < NDIR; ++k)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int col = cg + CPI * q;
      ev[k][q] = ld_coh(v + nbs[k] * NC + col);
#pragma unroll
      for (int i = 0; i < R; ++i) yv[k][q][i] = Ys[(long)k * NC * NC + col * NC + i];
    }
#pragma unroll
  for (int i = 0; i < R; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll
  for (int k = 0; k < NDIR; ++k)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int i = 0; i < R; ++i) cfma<T>(acc[i], yv[k][q][i], ev[k][q]);
#pragma unroll
  for (int i = 0; i < R; ++i) {
#pragma unroll
    for (int o = LPC; o < 64; o <<= 1) {
      acc[i].x += __shfl_xor(acc[i].x, o, 64);
      acc[i].y += __shfl_xor(acc[i].y, o, 64);
    }
  }
}

template <typename T, int NDIR>
__global__ __launch_bounds__(PG_THREADS) void gcr16_persistent_kernel(PgArgs<T> a) {
  constexpr int NC = 16;
  constexpr int R = (sizeof(T) == 4) ? 2 : 1;
  constexpr int LPC = NC / R;
  __shared__ double sh[PG_WAVES][PG_NQ];  // per-wave partial sums
  __shared__ double tot[PG_NQ];
  __shared__ double wwh[GCR_KMAX];
  __shared__ double coef[2 * GCR_KMAX + 2];
  const int rhs = blockIdx.y;
  const int blk = blockIdx.x;
  const unsigned nblk = gridDim.x;
  const long V = a.g.V;
  const long n = V * NC;
  const long ro = (long)rhs * n;
  gptr<const cplx<T>> b = gl(a.b) + ro;
  cplx<T>* x = a.x + ro;  // agent-coherent accesses only
  cplx<T>* r = a.r + ro;  // agent-coherent accesses only
  gptr<const cplx<T>> Y = gl(a.Y);
  unsigned* bar = a.bar + rhs;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = lane / LPC, rg = lane - cg * LPC;
  const bool own = cg == 0;
  const long s0 = (long)blk * PG_WAVES + wave, sstride = (long)nblk * PG_WAVES;
  double* part0 = a.part + (long)rhs * 2 * nblk * PG_NQ;
  const long half = (long)nblk * PG_NQ;
  unsigned pub = 0, epoch = 0;

  auto clear = [&]() {
    for (int q = threadIdx.x; q < PG_WAVES * PG_NQ; q += PG_THREADS) (&sh[0][0])[q] = 0.0;
    __syncthreads();
  };
  // add a value of every lane to the wave's slot q (whole wave active)
  auto wave_add = [&](int q, double v) {
    v = wave_sum(v);
    if (lane == 0) sh[wave][q] += v;
  };
  // block partials -> published -> barrier -> totals of all blocks in tot[0..nq)
  auto reduce = [&](int nq) {
    __syncthreads();
    double* part = part0 + (pub & 1u) * half;
    for (int q = threadIdx.x; q < nq; q += PG_THREADS) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < PG_WAVES; ++w) s += sh[w][q];
      __hip_atomic_store(&part[(long)blk * PG_NQ + q], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_barrier(bar, nblk, epoch, a.err);
    for (int q = threadIdx.x; q < nq; q += PG_THREADS) {
      double s = 0.0;
#pragma unroll 8
      for (unsigned bk = 0; bk < nblk; ++bk)
        s += __hip_atomic_load(&part[(long)bk * PG_NQ + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tot[q] = s;
    }
    pub += 1;
    __syncthreads();
  };

  // x = 0, r = b, bb = <b, b>
  clear();
  for (long site = s0; site < V; site += sstride) {
    double s = 0.0;
    if (own)
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const long idx = site * NC + rg * R + i;
        const cplx<T> v = b[idx];
        st_coh(x + idx, mk<T>(0, 0));
        st_coh(r + idx, v);
        s += (double)v.x * v.x + (double)v.y * v.y;
      }
    wave_add(0, s);
  }
  reduce(1);
  const double bb = tot[0];
  bool done = (a.tol2 >= 1.0) ? true : (bb == 0.0);
  int it = 0;
  for (; it < a.maxiter && !done; ++it) {
    const int k = it % a.m;
    if (k == 0 && it > 0) {
      // restart: r = b - A x
      for (long site = s0; site < V; site += sstride) {
        cplx<T> acc[R];
        pg_apply<T, NDIR>(Y, a.g, x, site, cg, rg, acc);
        if (own)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const long idx = site * NC + rg * R + i;
            st_coh(r + idx, csub<T>(b[idx], acc[i]));
          }
      }
      grid_barrier(bar, nblk, epoch, a.err);
    }
    gptr<cplx<T>> Wk = gl(a.Wb) + (long)k * a.dstride + ro;
    gptr<cplx<T>> Zk = gl(a.Zb) + (long)k * a.dstride + ro;
    // w = A r (stored as W_k), z = r (Z_k), dots <W_j, w> (j < k)
    clear();
    for (long site = s0; site < V; site += sstride) {
      cplx<T> acc[R];
      pg_apply<T, NDIR>(Y, a.g, r, site, cg, rg, acc);
      if (own)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const long idx = site * NC + rg * R + i;
          Wk[idx] = acc[i];
          Zk[idx] = ld_coh(r + idx);
        }
      for (int j = 0; j < k; ++j) {
        double dr = 0.0, di = 0.0;
        if (own) {
          gptr<const cplx<T>> Wj = gl(a.Wb) + (long)j * a.dstride + ro + site * NC + rg * R;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const cplx<T> q = Wj[i];
            dr += (double)q.x * acc[i].x + (double)q.y * acc[i].y;
            di += (double)q.x * acc[i].y - (double)q.y * acc[i].x;
          }
        }
        wave_add(2 * j, dr);
        wave_add(2 * j + 1, di);
      }
    }
    reduce(2 * k);
    for (int j = threadIdx.x; j < k; j += PG_THREADS) {
      const double s = wwh[j] > 0.0 ? 1.0 / wwh[j] : 0.0;
      coef[2 * j] = tot[2 * j] * s;
      coef[2 * j + 1] = tot[2 * j + 1] * s;
    }
    __syncthreads();
    // w -= sum beta_j W_j, z -= sum beta_j Z_j; <w,w>, <w,r>
    clear();
    for (long site = s0; site < V; site += sstride) {
      double s0w = 0.0, s1 = 0.0, s2 = 0.0;
      if (own)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const long idx = site * NC + rg * R + i;
          cplx<T> wi = Wk[idx], zi = Zk[idx];
          for (int j = 0; j < k; ++j) {
            const cplx<T> bj = mk<T>((T)coef[2 * j], (T)coef[2 * j + 1]);
            wi = csub<T>(wi, cmul<T>(bj, gl(a.Wb)[(long)j * a.dstride + ro + idx]));
            zi = csub<T>(zi, cmul<T>(bj, gl(a.Zb)[(long)j * a.dstride + ro + idx]));
          }
          if (k > 0) { Wk[idx] = wi; Zk[idx] = zi; }
          const cplx<T> ri = ld_coh(r + idx);
          s0w += (double)wi.x * wi.x + (double)wi.y * wi.y;
          s1 += (double)wi.x * ri.x + (double)wi.y * ri.y;
          s2 += (double)wi.x * ri.y - (double)wi.y * ri.x;
        }
      wave_add(0, s0w);
      wave_add(1, s1);
      wave_add(2, s2);
    }
    reduce(3);
    if (threadIdx.x == 0) {
      const double ww = tot[0];
      wwh[k] = ww;
      const double s = ww > 0.0 ? 1.0 / ww : 0.0;
      coef[2 * GCR_KMAX] = tot[1] * s;
      coef[2 * GCR_KMAX + 1] = tot[2] * s;
    }
    __syncthreads();
    // x += alpha z, r -= alpha w, <r, r>
    clear();
    {
      const cplx<T> al = mk<T>((T)coef[2 * GCR_KMAX], (T)coef[2 * GCR_KMAX + 1]);
      for (long site = s0; site < V; site += sstride) {
        double s = 0.0;
        if (own)
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const long idx = site * NC + rg * R + i;
            st_coh(x + idx, cadd<T>(ld_coh(x + idx), cmul<T>(al, Zk[idx])));
            const cplx<T> ri = csub<T>(ld_coh(r + idx), cmul<T>(al, Wk[idx]));
            st_coh(r + idx, ri);
            s += (double)ri.x * ri.x + (double)ri.y * ri.y;
          }
        wave_add(0, s);
      }
    }
    reduce(1);
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
  if (g.nd != 2 && g.nd != 4) return hipErrorInvalidValue;
  const void* fn = (g.nd == 2) ? (const void*)gcr16_persistent_kernel<T, 5> : (const void*)gcr16_persistent_kernel<T, 9>;
  if (cooperative) {
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)nblk, (unsigned)nrhs), dim3(PG_THREADS), args, 0, st);
  }
  // plain launch: the grid is at most one block per compute unit, and the
  // bounded barrier wait ends the kernel with an error flag should a block
  // ever not be resident
  if (g.nd == 2)
    hipLaunchKernelGGL((gcr16_persistent_kernel<T, 5>), dim3((unsigned)nblk, (unsigned)nrhs), dim3(PG_THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((gcr16_persistent_kernel<T, 9>), dim3((unsigned)nblk, (unsigned)nrhs), dim3(PG_THREADS), 0, st, a);
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

// Coarse-level kernels: the Galerkin block stencil (Eq. (2) applied to D),
// block restriction / prolongation onto chirally split near-null vectors
// (Eq. (5) and the construction of v_{sj}), and the setup-side helpers
// (block orthonormalisation, Galerkin assembly).
//
// Coarse fields: [rhs][site][t], t = chi * N_v + k.  Coarse operator:
// Y[site][k][col][row], k = 0 the diagonal block, k = 1 + 2 mu the coupling
// to site + mu, k = 2 + 2 mu to site - mu; each block stored column-major so
// that the threads of one site (one per row) read consecutive addresses.
// D_hat^dagger = Gamma_5 D_hat Gamma_5 with Gamma_5 = diag(+1_{N_v}, -1_{N_v})
// because P commutes with gamma_5.
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "dispatch.h"

namespace amg {
namespace {

__device__ __forceinline__ void coords(long site, const int (&dims)[4], int nd, int (&x)[4]) {
  long rem = site;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    x[mu] = 0;
    if (mu < nd) { x[mu] = (int)(rem % dims[mu]); rem /= dims[mu]; }
  }
}

__device__ __forceinline__ long neighbour(long site, const int (&x)[4], const int (&dims)[4], int nd, int dir) {
  // dir = 2 mu (+mu) or 2 mu + 1 (-mu)
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

template <typename T, int NC, int DAG, int EPI>
__global__ __launch_bounds__(256) void coarse_kernel(CoarseArgs<T> a0, const CoarseArgs<T>* batch) {
  AMG_ARGS(CoarseArgs<T>)
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const int nc = NC > 0 ? NC : a.g.nc;
  const int nd = a.g.nd;
  const int ndir = 2 * nd + 1;
  const long V = a.g.V;
  const long total = V * nc;
  const long ro = (long)rhs * total;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ Y = gl(a.Y);
  double acc3[3] = {0.0, 0.0, 0.0};
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long site = i / nc;
    const int row = (int)(i - site * nc);
    int x[4];
    coords(site, a.g.dims, nd, x);
    cplx<T> acc = mk<T>(0, 0);
    for (int k = 0; k < ndir; ++k) {
      const long nb = (k == 0) ? site : neighbour(site, x, a.g.dims, nd, k - 1);
      gptr<const cplx<T>> __restrict__ Yk = Y + ((site * ndir + k) * nc) * (long)nc + row;
      gptr<const cplx<T>> __restrict__ e = pin + nb * nc;
      if (NC > 0 && NC <= 16) {
        // all loads of the direction in flight at once
        cplx<T> ev[NC > 0 && NC <= 16 ? NC : 1], yv[NC > 0 && NC <= 16 ? NC : 1];
#pragma unroll
        for (int col = 0; col < NC; ++col) {
          ev[col] = e[col];
          yv[col] = Yk[(long)col * NC];
        }
#pragma unroll
        for (int col = 0; col < NC; ++col) {
          cplx<T> v = ev[col];
          if (DAG && col >= NC / 2) v = mk<T>(-v.x, -v.y);
          cfma<T>(acc, yv[col], v);
        }
      } else {
#pragma unroll 4
        for (int col = 0; col < nc; ++col) {
          cplx<T> v = e[col];
          if (DAG && col >= nc / 2) v = mk<T>(-v.x, -v.y);
          cfma<T>(acc, Yk[(long)col * nc], v);
        }
      }
    }
    if (DAG && row >= nc / 2) acc = mk<T>(-acc.x, -acc.y);
    const cplx<T> c = pin[i];
    if (EPI == EPI_RESID) acc = csub<T>(gl(a.b)[ro + i], acc);
    gl(a.out)[ro + i] = acc;
    if (a.copy_out) gl(a.copy_out)[ro + i] = c;
    if (EPI == EPI_MRDOT) {
      acc3[0] += (double)acc.x * c.x + (double)acc.y * c.y;
      acc3[1] += (double)acc.x * c.y - (double)acc.y * c.x;
      acc3[2] += (double)acc.x * acc.x + (double)acc.y * acc.y;
    } else if (EPI == EPI_NORM) {
      acc3[0] += (double)acc.x * acc.x + (double)acc.y * acc.y;
    }
  }
  if (EPI == EPI_MRDOT) {
    double tot[3];
    if (grid_reduce<3>(acc3, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) finalize_mr(tot, a.red, rhs);
  } else if (EPI == EPI_NORM) {
    double a1[1] = {acc3[0]}, tot[1];
    if (grid_reduce<1>(a1, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) a.red.scal[a.red.slot + rhs] = tot[0];
  }
}

// Wave-per-site variant for N_c = 16 (the 2d hierarchy).  The blocks of a
// site (16 columns of 16 rows per direction, contiguous) are streamed with
// each lane loading 16 bytes: R = 16 / sizeof(complex T) rows of one column
// per lane, LPC = 16 / R lanes per column, CPI = 64 / LPC columns per load.
// All loads of one direction are issued before its multiply-adds; partial
// row sums are then reduced across the lanes that share the rows, leaving
// the 16 results in lanes 0 .. LPC-1.
template <typename T> struct C16 {
  static constexpr int NC = 16;
  static constexpr int R = (sizeof(T) == 4) ? 2 : 1;
  static constexpr int LPC = NC / R;
  static constexpr int CPI = 64 / LPC;
  static constexpr int NQ = NC / CPI;  // loads per lane per direction
};

// ND = 2: the five directions are known at compile time, so the loads of all
// of them are issued before the first multiply-add (one memory round trip per
// site instead of five: the 2d coarse levels are small and latency-bound).
// ND = 0: any dimension, one direction at a time.
template <typename T, int DAG, int ND>
__device__ __forceinline__ void site_apply16(gptr<const cplx<T>> __restrict__ Y, gptr<const cplx<T>> __restrict__ pin, long site,
                                             const CoarseGeom& g, int cg, int rg, cplx<T> (&acc)[C16<T>::R]) {
  using K = C16<T>;
#pragma unroll
  for (int i = 0; i < K::R; ++i) acc[i] = mk<T>(0, 0);
  if (ND == 2) {
    constexpr int NDIR = 5;
    const int L1 = g.dims[0], L2 = g.dims[1];
    const int x1 = (int)(site % L1), x2 = (int)(site / L1);
    long nbs[NDIR];
    nbs[0] = site;
    nbs[1] = (x1 == L1 - 1) ? site - (L1 - 1) : site + 1;
    nbs[2] = (x1 == 0) ? site + (L1 - 1) : site - 1;
    nbs[3] = (x2 == L2 - 1) ? site - (long)(L2 - 1) * L1 : site + L1;
    nbs[4] = (x2 == 0) ? site + (long)(L2 - 1) * L1 : site - L1;
    gptr<const cplx<T>> __restrict__ Ys = Y + site * (long)NDIR * K::NC * K::NC + rg * K::R;
    cplx<T> ev[NDIR][K::NQ], yv[NDIR][K::NQ][K::R];
#pragma unroll
    for (int k = 0; k < NDIR; ++k)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        ev[k][q] = pin[nbs[k] * K::NC + col];
#pragma unroll
        for (int i = 0; i < K::R; ++i) yv[k][q][i] = Ys[(long)k * K::NC * K::NC + col * K::NC + i];
      }
#pragma unroll
    for (int k = 0; k < NDIR; ++k)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        cplx<T> v = ev[k][q];
        if (DAG && col >= K::NC / 2) v = mk<T>(-v.x, -v.y);
#pragma unroll
        for (int i = 0; i < K::R; ++i) cfma<T>(acc[i], yv[k][q][i], v);
      }
  } else {
    int x[4];
    coords(site, g.dims, g.nd, x);
    const int ndir = 2 * g.nd + 1;
    gptr<const cplx<T>> __restrict__ Ys = Y + site * (long)ndir * K::NC * K::NC;
    for (int k = 0; k < ndir; ++k) {
      const long nb = (k == 0) ? site : neighbour(site, x, g.dims, g.nd, k - 1);
      gptr<const cplx<T>> __restrict__ e = pin + nb * K::NC;
      gptr<const cplx<T>> __restrict__ yk = Ys + (long)k * K::NC * K::NC + rg * K::R;
      cplx<T> ev[K::NQ], yv[K::NQ][K::R];
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        ev[q] = e[col];
#pragma unroll
        for (int i = 0; i < K::R; ++i) yv[q][i] = yk[col * K::NC + i];
      }
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        cplx<T> v = ev[q];
        if (DAG && col >= K::NC / 2) v = mk<T>(-v.x, -v.y);
#pragma unroll
        for (int i = 0; i < K::R; ++i) cfma<T>(acc[i], yv[q][i], v);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < K::R; ++i) {
#pragma unroll
    for (int o = K::LPC; o < 64; o <<= 1) {
      acc[i].x += __shfl_xor(acc[i].x, o, 64);
      acc[i].y += __shfl_xor(acc[i].y, o, 64);
    }
  }
}

template <typename T, int DAG, int EPI, int ND>
__global__ __launch_bounds__(256) void coarse16_kernel(CoarseArgs<T> a0, const CoarseArgs<T>* batch) {
  AMG_ARGS(CoarseArgs<T>)
  using K = C16<T>;
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long V = a.g.V;
  const long ro = (long)rhs * V * K::NC;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + ro;
  gptr<const cplx<T>> __restrict__ pb = gl(a.b) + ro;
  gptr<cplx<T>> __restrict__ pout = gl(a.out) + ro;
  gptr<cplx<T>> __restrict__ pcopy = gl(a.copy_out) + ro;
  const bool copy = a.copy_out != nullptr;
  const int lane = threadIdx.x & 63;
  const int cg = lane / K::LPC, rg = lane - cg * K::LPC;
  const int wave = threadIdx.x >> 6;
  double acc3[3] = {0.0, 0.0, 0.0};
  for (long site = (long)blockIdx.x * 4 + wave; site < V; site += (long)gridDim.x * 4) {
    // this lane's rows of the input (MR sums, copy) and of b, loaded with the stencil's operands
    const long o = site * K::NC + rg * K::R;
    cplx<T> c[K::R], bv[K::R];
#pragma unroll
    for (int i = 0; i < K::R; ++i) {
      c[i] = mk<T>(0, 0);
      bv[i] = mk<T>(0, 0);
      if (cg == 0 && (EPI == EPI_MRDOT || EPI == EPI_MRPART || copy)) c[i] = pin[o + i];
      if (cg == 0 && EPI == EPI_RESID) bv[i] = pb[o + i];
    }
    cplx<T> acc[K::R];
    site_apply16<T, DAG, ND>(gl(a.Y), pin, site, a.g, cg, rg, acc);
    if (cg == 0) {
#pragma unroll
      for (int i = 0; i < K::R; ++i) {
        const int row = rg * K::R + i;
        cplx<T> v = acc[i];
        if (DAG && row >= K::NC / 2) v = mk<T>(-v.x, -v.y);
        if (EPI == EPI_RESID) v = csub<T>(bv[i], v);
        pout[o + i] = v;
        if (copy) pcopy[o + i] = c[i];
        if (EPI == EPI_MRDOT || EPI == EPI_MRPART) {
          acc3[0] += (double)v.x * c[i].x + (double)v.y * c[i].y;
          acc3[1] += (double)v.x * c[i].y - (double)v.y * c[i].x;
          acc3[2] += (double)v.x * v.x + (double)v.y * v.y;
        } else if (EPI == EPI_NORM) {
          acc3[0] += (double)v.x * v.x + (double)v.y * v.y;
        }
      }
    }
  }
  if (EPI == EPI_MRPART) block_partials<3>(acc3, a.red.part, rhs);
  if (EPI == EPI_MRDOT) {
    double tot[3];
    if (grid_reduce<3>(acc3, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) finalize_mr(tot, a.red, rhs);
  } else if (EPI == EPI_NORM) {
    double a1[1] = {acc3[0]}, tot[1];
    if (grid_reduce<1>(a1, a.red.part, a.red.ticket, rhs, tot) && threadIdx.x == 0) a.red.scal[a.red.slot + rhs] = tot[0];
  }
}

// GCR step, part 1 (N_c = 16): w = A z for every site, stored raw, with the
// sums c_j = <W_j, w> (j < k), <w, w> and <w, r> accumulated on the way.  The
// last block forms beta_j = c_j / <W_j, W_j>, the norm of the orthogonalised
// direction <w', w'> = <w, w> - sum_j |c_j|^2 / <W_j, W_j> (the stored W_j
// are mutually orthogonal) and alpha = <w', r> / <w', w'> with
// <w', r> = <w, r> (the residual is orthogonal to every stored W_j).
// Algebraically this is the GCR step; it needs one reduction instead of two.
constexpr int G16_NQ = 2 * GCR_KMAX + 2;
template <typename T>
struct G16Args {
  CoarseArgs<T> c;
  const cplx<T>* r;
  const cplx<T>* Wb;
  long dstride;
  int k, beta_slot, ww_slot, alpha_slot;
  int nrhs;
};
template <typename T>
__global__ __launch_bounds__(256) void gcr16_apply_dots_kernel(G16Args<T> a0, const G16Args<T>* batch) {
  AMG_PICK(ga, G16Args<T>)
  if ((int)blockIdx.y >= ga.nrhs) return;
  const CoarseArgs<T>& a = ga.c;
  const cplx<T>* __restrict__ r = ga.r;
  const cplx<T>* __restrict__ Wb = ga.Wb;
  const long dstride = ga.dstride;
  const int k = ga.k, beta_slot = ga.beta_slot, ww_slot = ga.ww_slot, alpha_slot = ga.alpha_slot;
  using K = C16<T>;
  __shared__ double sh[4 * K::LPC * G16_NQ];
  __shared__ double blk_part[G16_NQ];
  __shared__ int is_last;
  const int rhs = blockIdx.y;
  if (skip_rhs(a.red.flags, rhs)) return;
  const long V = a.g.V;
  const long ro = (long)rhs * V * K::NC;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = lane / K::LPC, rg = lane - cg * K::LPC;
  const int nq = 2 * k + 2;
  for (int q = threadIdx.x; q < 4 * K::LPC * G16_NQ; q += blockDim.x) sh[q] = 0.0;
  __syncthreads();
  double* mine = sh + (wave * K::LPC + rg) * G16_NQ;  // this lane's accumulators (cg == 0 lanes)
  for (long site = (long)blockIdx.x * 4 + wave; site < V; site += (long)gridDim.x * 4) {
    cplx<T> acc[K::R];
    if (a.g.nd == 2) site_apply16<T, 0, 2>(gl(a.Y), gl(a.in) + ro, site, a.g, cg, rg, acc);
    else site_apply16<T, 0, 0>(gl(a.Y), gl(a.in) + ro, site, a.g, cg, rg, acc);
    if (cg == 0) {
      double ww = 0.0, wrr = 0.0, wri = 0.0;
#pragma unroll
      for (int i = 0; i < K::R; ++i) {
        const long idx = ro + site * K::NC + rg * K::R + i;
        const cplx<T> w = acc[i];
        a.out[idx] = w;
        const cplx<T> rv = r[idx];
        ww += (double)w.x * w.x + (double)w.y * w.y;
        wrr += (double)w.x * rv.x + (double)w.y * rv.y;
        wri += (double)w.x * rv.y - (double)w.y * rv.x;
      }
      mine[2 * k] += ww;
      mine[2 * k + 1] += 0.0;
      for (int j = 0; j < k; ++j) {
        const cplx<T>* Wj = Wb + (long)j * dstride + ro + site * K::NC + rg * K::R;
        double cr = 0.0, ci = 0.0;
#pragma unroll
        for (int i = 0; i < K::R; ++i) {
          const cplx<T> q = Wj[i], w = acc[i];
          cr += (double)q.x * w.x + (double)q.y * w.y;
          ci += (double)q.x * w.y - (double)q.y * w.x;
        }
        mine[2 * j] += cr;
        mine[2 * j + 1] += ci;
      }
      // <w, r> in the spare slots after the dots
      mine[2 * k + 1] += wrr;
      mine[G16_NQ - 1] += wri;
    }
  }
  __syncthreads();
  const int nblk = gridDim.x;
  for (int q = threadIdx.x; q < G16_NQ; q += blockDim.x) {
    if (q < nq || q == G16_NQ - 1) {
      double s = 0.0;
      for (int l = 0; l < 4 * K::LPC; ++l) s += sh[l * G16_NQ + q];
      __hip_atomic_store(&a.red.part[((long)rhs * G16_NQ + q) * nblk + blockIdx.x], s, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  // partials published as in grid_reduce: agent-scope atomic stores, complete
  // before the ticket is taken, read back with agent-scope atomic loads
  wait_stores_complete();
  __syncthreads();
  if (threadIdx.x == 0)
    is_last = last_block(a.red.ticket, rhs);
  __syncthreads();
  if (!is_last) return;
  // every thread sums a stride of the blocks for each quantity, then the
  // waves are combined: loads stay independent and the order fixed
  __shared__ double wsum[4][G16_NQ];
  for (int q = 0; q < G16_NQ; ++q) {
    if (!(q < nq || q == G16_NQ - 1)) continue;
    double s = 0.0;
    for (int bk = threadIdx.x; bk < nblk; bk += blockDim.x)
      s += __hip_atomic_load(&a.red.part[((long)rhs * G16_NQ + q) * nblk + bk], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) wsum[wave][q] = s;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < G16_NQ; q += blockDim.x)
    blk_part[q] = (q < nq || q == G16_NQ - 1) ? (wsum[0][q] + wsum[1][q]) + (wsum[2][q] + wsum[3][q]) : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* scal = a.red.scal;
    double wwp = blk_part[2 * k];
    for (int j = 0; j < k; ++j) {
      const double wwj = scal[ww_slot + rhs * GCR_KMAX + j];
      const double s = wwj > 0.0 ? 1.0 / wwj : 0.0;
      const double cr = blk_part[2 * j], ci = blk_part[2 * j + 1];
      scal[beta_slot + (rhs * GCR_KMAX + j) * 2] = cr * s;
      scal[beta_slot + (rhs * GCR_KMAX + j) * 2 + 1] = ci * s;
      wwp -= (cr * cr + ci * ci) * s;
    }
    scal[ww_slot + rhs * GCR_KMAX + k] = wwp;
    const double s = wwp > 0.0 ? 1.0 / wwp : 0.0;
    scal[alpha_slot + 2 * rhs] = blk_part[2 * k + 1] * s;
    scal[alpha_slot + 2 * rhs + 1] = blk_part[G16_NQ - 1] * s;
  }
}

// Split apply (FP64) of a coarse operator for the next Galerkin product:
// out[0] = diagonal + hops inside the next block, out[1 + dir] = the hop in
// direction dir when it leaves the block through its face.
__global__ __launch_bounds__(256) void coarse_split_kernel(double2* __restrict__ out, const double2* __restrict__ in,
                                                           const double2* __restrict__ Y, CoarseGeom g,
                                                           int b0, int b1, int b2, int b3, int nrhs) {
  const int rhs = blockIdx.y;
  const int nc = g.nc, nd = g.nd, ndir = 2 * nd + 1;
  const int blk[4] = {b0, b1, b2, b3};
  const long total = g.V * nc;
  const long ro = (long)rhs * total;
  const long kstride = (long)nrhs * total;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long site = i / nc;
    const int row = (int)(i - site * nc);
    int x[4];
    coords(site, g.dims, nd, x);
    double2 inner = mk<double>(0, 0);
    for (int k = 0; k < ndir; ++k) {
      const long nb = (k == 0) ? site : neighbour(site, x, g.dims, nd, k - 1);
      const double2* Yk = Y + ((site * ndir + k) * nc) * (long)nc + row;
      const double2* e = in + ro + nb * nc;
      double2 acc = mk<double>(0, 0);
      for (int col = 0; col < nc; ++col) cfma<double>(acc, Yk[(long)col * nc], e[col]);
      bool cross = false;
      if (k > 0) {
        const int mu = (k - 1) >> 1;
        const int face = ((k - 1) & 1) ? 0 : at4(blk, mu) - 1;
        cross = (at4(x, mu) % at4(blk, mu)) == face;
      }
      if (cross) {
        out[(long)k * kstride + ro + i] = acc;
      } else {
        inner = cadd<double>(inner, acc);
        if (k > 0) out[(long)k * kstride + ro + i] = mk<double>(0, 0);
      }
    }
    out[ro + i] = inner;
  }
}

__global__ __launch_bounds__(256) void coarse_massmat_kernel(double2* __restrict__ out, const double2* __restrict__ in,
                                                             const double2* __restrict__ M, long V, int nc) {
  const int rhs = blockIdx.y;
  const long total = V * nc;
  const long ro = (long)rhs * total;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long site = i / nc;
    const int row = (int)(i - site * nc);
    const double2* Ms = M + site * (long)nc * nc + row;
    const double2* e = in + ro + site * nc;
    double2 acc = mk<double>(0, 0);
    for (int col = 0; col < nc; ++col) cfma<double>(acc, Ms[(long)col * nc], e[col]);
    out[ro + i] = acc;
  }
}

// ---- transfers ---------------------------------------------------------------

struct BlockIdx {
  // fine site of (coarse site j, site-in-block xi)
  // (32-bit index arithmetic: lattices have fewer than 2^31 sites)
  static __device__ __forceinline__ long fine_site(const TransferGeom& g, long j, int xi) {
    int rj = (int)j;
    int rxi = xi;
    int fs = 0, stride = 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if (mu < g.nd) {
        const int jc = rj % g.cdims[mu]; rj /= g.cdims[mu];
        const int bc = rxi % g.blk[mu]; rxi /= g.blk[mu];
        fs += (jc * g.blk[mu] + bc) * stride;
        stride *= g.fdims[mu];
      }
    }
    return fs;
  }
  // (coarse site, site-in-block) of a fine site
  static __device__ __forceinline__ void coarse_of(const TransferGeom& g, long fs, long& j, int& xi) {
    int rem = (int)fs, cs = 1, jj = 0;
    int bstride = 1;
    xi = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if (mu < g.nd) {
        const int x = rem % g.fdims[mu]; rem /= g.fdims[mu];
        jj += (x / g.blk[mu]) * cs;
        xi += (x % g.blk[mu]) * bstride;
        cs *= g.cdims[mu];
        bstride *= g.blk[mu];
      }
    }
    j = jj;
  }
};

template <typename T, typename PT>
struct TrArgs {
  cplx<T>* out;
  const cplx<T>* in;
  const PT* P;
  TransferGeom g;
  const int* flags;
  int accumulate;
  int nrhs;
};

template <typename T, typename PT>
__global__ __launch_bounds__(256) void restrict_kernel(TrArgs<T, PT> a0, const TrArgs<T, PT>* batch) {
  AMG_ARGS(TrArgs<T, PT>)
  const TransferGeom& g = a.g;
  gptr<cplx<T>> __restrict__ out = gl(a.out);
  gptr<const cplx<T>> __restrict__ in = gl(a.in);
  gptr<const PT> __restrict__ P = gl(a.P);
  const int rhs = blockIdx.y;
  if (skip_rhs(a.flags, rhs)) return;
  const int nc = 2 * g.nv, hd = g.dof / 2;
  const long total = g.Vc * nc;
  const long rof = (long)rhs * g.lf.per_rhs();
  const long roc = (long)rhs * total;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long j = i / nc;
    const int t = (int)(i - j * nc);
    const int chi = t / g.nv, k = t - chi * g.nv;
    cplx<T> acc = mk<T>(0, 0);
    for (int xi = 0; xi < g.bs; ++xi) {
      const long fs = BlockIdx::fine_site(g, j, xi);
      const long pb = ((j * g.bs + xi) * g.dof) * (long)g.nv + k;
      for (int h = 0; h < hd; ++h) {
        const int comp = chi * hd + h;
        cjfma<T>(acc, ldp<T>(P, pb + (long)comp * g.nv), in[rof + g.lf.off(fs, comp)]);
      }
    }
    out[roc + i] = acc;
  }
}

template <typename T, typename PT>
__global__ __launch_bounds__(256) void prolong_kernel(TrArgs<T, PT> a0, const TrArgs<T, PT>* batch) {
  AMG_ARGS(TrArgs<T, PT>)
  const TransferGeom& g = a.g;
  gptr<cplx<T>> __restrict__ out = gl(a.out);
  gptr<const cplx<T>> __restrict__ in = gl(a.in);
  gptr<const PT> __restrict__ P = gl(a.P);
  const int accumulate = a.accumulate;
  const int rhs = blockIdx.y;
  if (skip_rhs(a.flags, rhs)) return;
  const int nc = 2 * g.nv, hd = g.dof / 2;
  const long total = g.Vf * g.dof;
  const long rof = (long)rhs * g.lf.per_rhs();
  const long roc = (long)rhs * g.Vc * nc;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    // i enumerates (component, site) with the site fastest so that stores of
    // the structure-of-arrays planes are contiguous
    const int comp = (int)(i / g.Vf);
    const long fs = i - (long)comp * g.Vf;
    long j; int xi;
    BlockIdx::coarse_of(g, fs, j, xi);
    const int chi = comp / hd;
    const long pb = ((j * g.bs + xi) * g.dof + comp) * (long)g.nv;
    gptr<const cplx<T>> e = in + roc + j * nc + chi * g.nv;
    cplx<T> acc = mk<T>(0, 0);
    for (int k = 0; k < g.nv; ++k) cfma<T>(acc, ldp<T>(P, pb + k), e[k]);
    const long o = rof + g.lf.off(fs, comp);
    out[o] = accumulate ? cadd<T>(out[o], acc) : acc;
  }
}

// ---- transfers for large blocks (4d: 256 sites x 6 components per chirality) --
// One wave per (coarse site j, chirality chi); right-hand sides go in groups
// of RG inside the wave, so every row of P is read once per group instead of
// once per right-hand side (the per-element kernels above re-read all of P
// for each rhs and serialise 1536 terms per thread).
//
// restriction: lane l < 2 NV owns coarse component k = l mod NV and the
// components h of parity l / NV; consecutive lanes read consecutive k of one
// row of P.  The two parities are combined by one cross-lane add.
template <typename T, typename PT, int NV, int RG>
__global__ __launch_bounds__(256) void restrict_blk_kernel(TrArgs<T, PT> a0, const TrArgs<T, PT>* batch) {
  AMG_ARGS(TrArgs<T, PT>)
  const TransferGeom& g = a.g;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long q = (long)blockIdx.x * 4 + wave;
  if (q >= g.Vc * 2) return;
  const long j = q >> 1;
  const int chi = (int)(q & 1);
  const int k = lane % NV, par = lane / NV;
  const bool active = lane < 2 * NV;
  const int hd = g.dof / 2;
  const long per_f = g.lf.per_rhs(), per_c = g.Vc * 2 * NV;
  // the fine values of a batch, loaded once by the whole wave: [parity][u][r]
  constexpr int UN = 6;
  __shared__ cplx<T> xs[4][2][UN][RG];
  const long fs0 = BlockIdx::fine_site(g, j, 0);
  const int s1 = g.fdims[0], s2 = s1 * g.fdims[1], s3 = s2 * g.fdims[2];
  const int nel0 = g.bs * ((hd + 1) / 2), nel1 = g.bs * (hd / 2);  // elements per parity
  // fine field offset of element e of parity p (sites of the block in P order)
  auto fine_off = [&](int p, int e) -> long {
    const int hn = p ? hd / 2 : (hd + 1) / 2;
    const int xi = e / hn, h = p + 2 * (e - xi * hn);
    int rem = xi;
    const int b0 = rem % g.blk[0]; rem /= g.blk[0];
    const int b1 = rem % g.blk[1]; rem /= g.blk[1];
    const int b2 = rem % g.blk[2]; rem /= g.blk[2];
    const long fs = fs0 + b0 + b1 * s1 + b2 * s2 + (long)rem * s3;
    return g.lf.off(fs, chi * hd + h);
  };
  const int pc = active ? par : 0;
  const int hn = pc ? hd / 2 : (hd + 1) / 2;  // components of this lane's parity per site
  const int nel = pc ? nel1 : nel0;
  const long pbase = (j * g.bs * g.dof + chi * hd) * (long)NV + k;
  for (int r0 = 0; r0 < a.nrhs; r0 += RG) {
    const int nr = (a.nrhs - r0 < RG) ? a.nrhs - r0 : RG;
    cplx<T> acc[RG];
#pragma unroll
    for (int r = 0; r < RG; ++r) acc[r] = mk<T>(0, 0);
    for (int e0 = 0; e0 < nel0; e0 += UN) {
      // every lane loads distinct fine values of the batch into LDS
      constexpr int NT = (2 * UN * RG + 63) / 64;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int v = lane + 64 * t;
        if (v < 2 * UN * RG) {
          const int p = v / (UN * RG), rest = v - p * (UN * RG);
          const int u = rest / RG, r = rest - u * RG;
          const int e = e0 + u;
          cplx<T> x = mk<T>(0, 0);
          if (r < nr && e < (p ? nel1 : nel0)) x = gl(a.in)[(long)(r0 + r) * per_f + fine_off(p, e)];
          xs[wave][p][u][r] = x;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (active) {
        cplx<T> pv[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
          const int e = (e0 + u < nel) ? e0 + u : nel - 1;
          const int xi = e / hn, h = par + 2 * (e - xi * hn);
          const T w = (e0 + u < nel) ? (T)1 : (T)0;
          const cplx<T> pp = ldp<T>(gl(a.P), pbase + ((long)xi * g.dof + h) * NV);
          pv[u] = mk<T>(w * pp.x, w * pp.y);
        }
#pragma unroll
        for (int r = 0; r < RG; ++r)
          if (r < nr)
#pragma unroll
            for (int u = 0; u < UN; ++u) cjfma<T>(acc[r], pv[u], xs[wave][par][u][r]);
      }
      // the next batch overwrites xs only after every lane has read this one
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      const int src = (lane + NV) & 63;
      const T ox = __shfl(acc[r].x, src, 64), oy = __shfl(acc[r].y, src, 64);
      if (r < nr && lane < NV && !skip_rhs(a.flags, r0 + r))
        gl(a.out)[(long)(r0 + r) * per_c + j * 2 * NV + chi * NV + k] = mk<T>(acc[r].x + ox, acc[r].y + oy);
    }
  }
}

// prolongation: lane owns (site xi, component pair hp) elements of the block
// (sites fastest, for the fine-field stores) and computes both components of
// the pair for RG right-hand sides; the coarse values of (j, chi) are read by
// every lane (cache broadcast).
template <typename T, typename PT, int NV, int RG>
__global__ __launch_bounds__(256) void prolong_blk_kernel(TrArgs<T, PT> a0, const TrArgs<T, PT>* batch) {
  AMG_ARGS(TrArgs<T, PT>)
  const TransferGeom& g = a.g;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long q = (long)blockIdx.x * 4 + wave;
  if (q >= g.Vc * 2) return;
  const long j = q >> 1;
  const int chi = (int)(q & 1);
  const int hd = g.dof / 2, hp_n = hd / 2;
  const long per_f = g.lf.per_rhs(), per_c = g.Vc * 2 * NV;
  const long fs0 = BlockIdx::fine_site(g, j, 0);
  const int s1 = g.fdims[0], s2 = s1 * g.fdims[1], s3 = s2 * g.fdims[2];
  // this wave's coarse values [rhs][k] (the same for all its lanes), staged
  // once per group of right-hand sides and read as LDS broadcasts
  __shared__ cplx<T> es[4][RG][NV];
  for (int r0 = 0; r0 < a.nrhs; r0 += RG) {
    const int nr = (a.nrhs - r0 < RG) ? a.nrhs - r0 : RG;
    {
      gptr<const cplx<T>> __restrict__ e = gl(a.in) + (long)r0 * per_c + j * 2 * NV + chi * NV;
      for (int v = lane; v < RG * NV; v += 64) {
        const int r = v / NV, k = v - r * NV;
        cplx<T> ev = mk<T>(0, 0);
        if (r < nr) ev = e[(long)r * per_c + k];
        es[wave][r][k] = ev;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    for (int xi = lane; xi < g.bs; xi += 64) {
      int rem = xi;
      const int b0 = rem % g.blk[0]; rem /= g.blk[0];
      const int b1 = rem % g.blk[1]; rem /= g.blk[1];
      const int b2 = rem % g.blk[2]; rem /= g.blk[2];
      const long fs = fs0 + b0 + b1 * s1 + b2 * s2 + (long)rem * s3;
      for (int hp = 0; hp < hp_n; ++hp) {
      const int c0 = chi * hd + 2 * hp;
      const long prow = ((j * g.bs + xi) * g.dof + c0) * (long)NV;
      cplx<T> s0[RG], s1[RG];  // (the pair's two components)
#pragma unroll
      for (int r = 0; r < RG; ++r) { s0[r] = mk<T>(0, 0); s1[r] = mk<T>(0, 0); }
      // the pair's P rows 16 bytes at a time (rows start 16-byte aligned: NV
      // entries of 4, 8 or 16 bytes with NV a multiple of 4)
      constexpr int QN = 16 / (int)sizeof(PT);
      for (int k0 = 0; k0 < NV; k0 += QN) {
        cplx<T> p0[QN], p1[QN];
        ldp16<T, PT>(gl(a.P) + prow + k0, p0);
        ldp16<T, PT>(gl(a.P) + prow + NV + k0, p1);
#pragma unroll
        for (int qq = 0; qq < QN; ++qq)
#pragma unroll
          for (int r = 0; r < RG; ++r)
            if (r < nr) {
              const cplx<T> ev = es[wave][r][k0 + qq];
              cfma<T>(s0[r], p0[qq], ev);
              cfma<T>(s1[r], p1[qq], ev);
            }
      }
      const long o0 = g.lf.off(fs, c0), o1 = g.lf.off(fs, c0 + 1);
#pragma unroll
      for (int r = 0; r < RG; ++r)
        if (r < nr && !skip_rhs(a.flags, r0 + r)) {
          gptr<cplx<T>> __restrict__ out = gl(a.out) + (long)(r0 + r) * per_f;
          out[o0] = a.accumulate ? cadd<T>(out[o0], s0[r]) : s0[r];
          out[o1] = a.accumulate ? cadd<T>(out[o1], s1[r]) : s1[r];
        }
      }
    }
    // the next group overwrites es only after every lane has read this one
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// One wave per (coarse site j, chirality chi): gather the block vectors into
// P and orthonormalise them by modified Gram-Schmidt applied twice, in vector
// order, with positive real normalisation.
__global__ __launch_bounds__(64) void orthonormalise_kernel(double2* __restrict__ P, const double2* __restrict__ vecs,
                                                            TransferGeom g, int* err) {
  const long j = blockIdx.x;
  const int chi = blockIdx.y;
  const int lane = threadIdx.x;
  const int hd = g.dof / 2, nv = g.nv;
  const int dim = g.bs * hd;
  const long per = g.lf.per_rhs();
  auto pidx = [&](int e, int k) -> long {
    const int xi = e / hd, h = e - xi * hd;
    return ((j * g.bs + xi) * g.dof + chi * hd + h) * (long)nv + k;
  };
  for (int k = 0; k < nv; ++k)
    for (int e = lane; e < dim; e += 64) {
      const int xi = e / hd, h = e - xi * hd;
      const long fs = BlockIdx::fine_site(g, j, xi);
      P[pidx(e, k)] = vecs[(long)k * per + g.lf.off(fs, chi * hd + h)];
    }
  for (int k = 0; k < nv; ++k) {
    double n0 = 0.0;
    for (int e = lane; e < dim; e += 64) { const double2 w = P[pidx(e, k)]; n0 += w.x * w.x + w.y * w.y; }
    n0 = sqrt(wave_sum(n0));
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < k; ++i) {
        double dr = 0.0, di = 0.0;
        for (int e = lane; e < dim; e += 64) {
          const double2 q = P[pidx(e, i)], w = P[pidx(e, k)];
          dr += q.x * w.x + q.y * w.y;
          di += q.x * w.y - q.y * w.x;
        }
        dr = wave_sum(dr); di = wave_sum(di);
        for (int e = lane; e < dim; e += 64) {
          const double2 q = P[pidx(e, i)];
          double2 w = P[pidx(e, k)];
          w.x -= dr * q.x - di * q.y;
          w.y -= dr * q.y + di * q.x;
          P[pidx(e, k)] = w;
        }
      }
    double nr = 0.0;
    for (int e = lane; e < dim; e += 64) { const double2 w = P[pidx(e, k)]; nr += w.x * w.x + w.y * w.y; }
    nr = sqrt(wave_sum(nr));
    if (!(nr > 1e-10 * n0) || n0 == 0.0) {
      if (lane == 0) *err = 1;
      nr = 1.0;
    }
    const double inv = 1.0 / nr;
    for (int e = lane; e < dim; e += 64) {
      double2 w = P[pidx(e, k)];
      w.x *= inv; w.y *= inv;
      P[pidx(e, k)] = w;
    }
  }
}

// Large blocks (more than 64 block elements per chirality, e.g. 4^4 sites x
// 6 components): classical Gram-Schmidt applied twice (CGS2), which gives the
// same orthonormal basis as the modified variant up to rounding.  Vector k
// stays in registers (EM elements per lane); each pass computes all the
// projections onto the finished vectors 0..k-1 at once, reading each row of
// P (its first k entries, contiguous) — no dependent memory round trips
// between the projections, as the modified variant has.  Positive real
// normalisation and the same rank test (remainder below 1e-10 of the
// original norm).
template <int EM, int NVM>
__global__ __launch_bounds__(64) void orthonormalise_cgs2_kernel(double2* __restrict__ P_,
                                                                 const double2* __restrict__ vecs_, TransferGeom g,
                                                                 int* err) {
  const long j = blockIdx.x;
  const int chi = blockIdx.y;
  const int lane = threadIdx.x;
  const int hd = g.dof / 2, nv = g.nv;
  const int dim = g.bs * hd;
  const long per = g.lf.per_rhs();
  gptr<double2> P = gl(P_) + j * g.bs * g.dof * (long)nv;  // this block's rows
  gptr<const double2> vecs = gl(vecs_);
  int row[EM];  // offsets of this lane's rows in the block
#pragma unroll
  for (int t = 0; t < EM; ++t) {
    const int e = lane + 64 * t;
    const int ec = e < dim ? e : dim - 1;
    const int xi = ec / hd, h = ec - xi * hd;
    row[t] = (xi * g.dof + chi * hd + h) * nv;
  }
  for (int k = 0; k < nv; ++k) {
    double2 w[EM];
    double n0 = 0.0;
#pragma unroll
    for (int t = 0; t < EM; ++t) {
      const int e = lane + 64 * t;
      w[t] = make_double2(0.0, 0.0);
      if (e < dim) {
        const int xi = e / hd, h = e - xi * hd;
        w[t] = vecs[(long)k * per + g.lf.off(BlockIdx::fine_site(g, j, xi), chi * hd + h)];
      }
      n0 += w[t].x * w[t].x + w[t].y * w[t].y;
    }
    n0 = sqrt(wave_sum(n0));
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      double cr[NVM], ci[NVM];
#pragma unroll
      for (int i = 0; i < NVM; ++i) { cr[i] = 0.0; ci[i] = 0.0; }
#pragma unroll
      for (int t = 0; t < EM; ++t) {
        if (lane + 64 * t < dim) {
#pragma unroll
          for (int i = 0; i < NVM; ++i)
            if (i < k) {
              const double2 q = P[row[t] + i];
              cr[i] += q.x * w[t].x + q.y * w[t].y;
              ci[i] += q.x * w[t].y - q.y * w[t].x;
            }
        }
      }
#pragma unroll
      for (int i = 0; i < NVM; ++i)
        if (i < k) {  // uniform
          cr[i] = wave_sum(cr[i]);
          ci[i] = wave_sum(ci[i]);
        }
#pragma unroll
      for (int t = 0; t < EM; ++t) {
        if (lane + 64 * t < dim) {
#pragma unroll
          for (int i = 0; i < NVM; ++i)
            if (i < k) {
              const double2 q = P[row[t] + i];
              w[t].x -= cr[i] * q.x - ci[i] * q.y;
              w[t].y -= cr[i] * q.y + ci[i] * q.x;
            }
        }
      }
    }
    double nr = 0.0;
#pragma unroll
    for (int t = 0; t < EM; ++t) nr += w[t].x * w[t].x + w[t].y * w[t].y;
    nr = sqrt(wave_sum(nr));
    if (!(nr > 1e-10 * n0) || n0 == 0.0) {
      if (lane == 0) *err = 1;
      nr = 1.0;
    }
    const double inv = 1.0 / nr;
#pragma unroll
    for (int t = 0; t < EM; ++t)
      if (lane + 64 * t < dim) P[row[t] + k] = make_double2(w[t].x * inv, w[t].y * inv);
  }
}

__global__ void galerkin_scatter_kernel(double2* __restrict__ Y, const double2* __restrict__ R, long Vc, int nc,
                                        int nk, int t0, int chunk) {
  const long total = (long)nk * chunk * Vc * nc;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    long r = i;
    const int t = (int)(r % nc); r /= nc;
    const long xs = r % Vc; r /= Vc;
    const int c = (int)(r % chunk); r /= chunk;
    const int k = (int)r;
    Y[((xs * nk + k) * nc + (t0 + c)) * (long)nc + t] = R[i];
  }
}

__global__ void unit_coarse_kernel(double2* __restrict__ E, long Vc, int nc, int t0, int chunk) {
  const long total = (long)chunk * Vc * nc;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int t = (int)(i % nc);
    const int c = (int)(i / ((long)Vc * nc));
    E[i] = mk<double>(t == t0 + c ? 1.0 : 0.0, 0.0);
  }
}

inline unsigned nblocks(long n, long cap = 1L << 20) {
  long b = (n + 255) / 256;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int coarse16_red_blocks(long V) {
  long nb = (V + 3) / 4;
  if (nb > red_block_cap()) nb = red_block_cap();
  return (int)nb;
}

template <typename T>
void launch_coarse(const CoarseArgs<T>& a, int dagger, int epi, hipStream_t st) {
  const long total = a.g.V * a.g.nc;
  const bool red = (epi == EPI_MRDOT || epi == EPI_NORM);
  dim3 grid(nblocks(total, red ? (long)red_block_cap() : (1L << 20)), (unsigned)a.nrhs);
#define AMG_C(NC, DAG, EPI) dispatch(coarse_kernel<T, NC, DAG, EPI>, a, grid, dim3(256), st)
#define AMG_C_EPI(NC, DAG)                      \
  switch (epi) {                                \
    case EPI_PLAIN: AMG_C(NC, DAG, EPI_PLAIN); break; \
    case EPI_MRDOT: AMG_C(NC, DAG, EPI_MRDOT); break; \
    case EPI_RESID: AMG_C(NC, DAG, EPI_RESID); break; \
    default: AMG_C(NC, DAG, EPI_NORM); break;   \
  }
  if (a.g.nc == 16) {
    long nb = (a.g.V + 3) / 4;
    const long cap = (red || epi == EPI_MRPART) ? (long)red_block_cap() : (1L << 20);
    if (nb > cap) nb = cap;
    dim3 g16((unsigned)nb, (unsigned)a.nrhs);
#define AMG_C16N(DAG, EPI, ND) dispatch(coarse16_kernel<T, DAG, EPI, ND>, a, g16, dim3(256), st)
#define AMG_C16(DAG, EPI) if (a.g.nd == 2) { AMG_C16N(DAG, EPI, 2); } else { AMG_C16N(DAG, EPI, 0); }
    switch (epi * 2 + (dagger ? 1 : 0)) {
      case EPI_PLAIN * 2: AMG_C16(0, EPI_PLAIN); break;
      case EPI_PLAIN * 2 + 1: AMG_C16(1, EPI_PLAIN); break;
      case EPI_MRDOT * 2: AMG_C16(0, EPI_MRDOT); break;
      case EPI_MRDOT * 2 + 1: AMG_C16(1, EPI_MRDOT); break;
      case EPI_RESID * 2: AMG_C16(0, EPI_RESID); break;
      case EPI_RESID * 2 + 1: AMG_C16(1, EPI_RESID); break;
      case EPI_NORM * 2: AMG_C16(0, EPI_NORM); break;
      case EPI_NORM * 2 + 1: AMG_C16(1, EPI_NORM); break;
      case EPI_MRPART * 2: AMG_C16(0, EPI_MRPART); break;
      default: AMG_C16(1, EPI_MRPART); break;
    }
#undef AMG_C16
#undef AMG_C16N
  } else if (a.g.nc == 48) {
    if (dagger) { AMG_C_EPI(48, 1) } else { AMG_C_EPI(48, 0) }
  } else if (std::is_same<T, double>::value && !dagger && (epi == EPI_PLAIN || epi == EPI_RESID) &&
             a.g.nc >= 2 && a.g.nc <= 14 && a.g.nc % 2 == 0) {
    // the partial hierarchies of the adaptive setup (2 .. 14 coarse dof, FP64)
#define AMG_CP(NC) \
  if (epi == EPI_RESID) { AMG_C(NC, 0, EPI_RESID); } else { AMG_C(NC, 0, EPI_PLAIN); }
    switch (a.g.nc) {
      case 2: AMG_CP(2) break;
      case 4: AMG_CP(4) break;
      case 6: AMG_CP(6) break;
      case 8: AMG_CP(8) break;
      case 10: AMG_CP(10) break;
      case 12: AMG_CP(12) break;
      default: AMG_CP(14) break;
    }
#undef AMG_CP
  } else {
    if (dagger) { AMG_C_EPI(0, 1) } else { AMG_C_EPI(0, 0) }
  }
#undef AMG_C_EPI
#undef AMG_C
}
template void launch_coarse<double>(const CoarseArgs<double>&, int, int, hipStream_t);
template void launch_coarse<float>(const CoarseArgs<float>&, int, int, hipStream_t);

template <typename T>
void launch_gcr16_apply_dots(const CoarseArgs<T>& a, const cplx<T>* r, const cplx<T>* Wb, long dstride, int k,
                             int beta_slot, int ww_slot, int alpha_slot, hipStream_t st) {
  long nb = (a.g.V + 3) / 4;
  if (nb > red_block_cap()) nb = red_block_cap();
  dim3 grid((unsigned)nb, (unsigned)a.nrhs);
  G16Args<T> ga{a, r, Wb, dstride, k, beta_slot, ww_slot, alpha_slot, a.nrhs};
  dispatch(gcr16_apply_dots_kernel<T>, ga, grid, dim3(256), st);
}
template void launch_gcr16_apply_dots<double>(const CoarseArgs<double>&, const double2*, const double2*, long, int,
                                              int, int, int, hipStream_t);
template void launch_gcr16_apply_dots<float>(const CoarseArgs<float>&, const float2*, const float2*, long, int, int,
                                             int, int, hipStream_t);

void launch_coarse_split(double2* out, const double2* in, const double2* Y, const CoarseGeom& g, const int* blk,
                         int nrhs, hipStream_t st) {
  dim3 grid(nblocks(g.V * g.nc), (unsigned)nrhs);
  hipLaunchKernelGGL(coarse_split_kernel, grid, dim3(256), 0, st, out, in, Y, g, blk[0], blk[1],
                     g.nd > 2 ? blk[2] : 1, g.nd > 3 ? blk[3] : 1, nrhs);
}

void launch_coarse_massmat(double2* out, const double2* in, const double2* M, const CoarseGeom& g, int nrhs,
                           hipStream_t st) {
  dim3 grid(nblocks(g.V * g.nc), (unsigned)nrhs);
  hipLaunchKernelGGL(coarse_massmat_kernel, grid, dim3(256), 0, st, out, in, M, g.V, g.nc);
}

// the per-wave kernels need an even number of components per chirality, a
// block large enough to fill a wave, and 2 NV <= 64 lanes
inline bool blk_transfer(const TransferGeom& g) {
  return g.nd == 4 && (g.dof / 2) % 2 == 0 && g.bs * (g.dof / 2) >= 512 && g.nv == 24;
}

template <typename T>
void launch_restrict(cplx<T>* out, const cplx<T>* in, const void* P, int pkind, const TransferGeom& g, int nrhs,
                     const int* flags, hipStream_t st) {
  // large blocks: the per-wave kernel, which reads P once per group of
  // right-hand sides (2x faster than the per-element kernel at 12 rhs, and
  // at one rhs the 4d one-rhs solve 1.14 -> 0.86 s with the prolongation)
  if (blk_transfer(g)) {
    const dim3 grid((unsigned)((g.Vc * 2 + 3) / 4), 1);
#define AMG_RB(PT, RG) dispatch(restrict_blk_kernel<T, PT, 24, RG>, TrArgs<T, PT>{out, in, (const PT*)P, g, flags, 0, nrhs}, grid, dim3(256), st)
#define AMG_RB_G(PT) if (nrhs == 1) { AMG_RB(PT, 1); } else if (nrhs <= 4) { AMG_RB(PT, 4); } else { AMG_RB(PT, 16); }
    if (pkind == P_F64) { AMG_RB_G(double2) }
    else if (pkind == P_F32) { AMG_RB_G(float2) }
    else { AMG_RB_G(bf16x2) }
#undef AMG_RB_G
#undef AMG_RB
    return;
  }
  dim3 grid(nblocks(g.Vc * 2 * g.nv), (unsigned)nrhs);
  if (pkind == P_F64)
    dispatch(restrict_kernel<T, double2>, TrArgs<T, double2>{out, in, (const double2*)P, g, flags, 0, nrhs}, grid, dim3(256), st);
  else if (pkind == P_F32)
    dispatch(restrict_kernel<T, float2>, TrArgs<T, float2>{out, in, (const float2*)P, g, flags, 0, nrhs}, grid, dim3(256), st);
  else
    dispatch(restrict_kernel<T, bf16x2>, TrArgs<T, bf16x2>{out, in, (const bf16x2*)P, g, flags, 0, nrhs}, grid, dim3(256), st);
}
template void launch_restrict<double>(double2*, const double2*, const void*, int, const TransferGeom&, int, const int*, hipStream_t);
template void launch_restrict<float>(float2*, const float2*, const void*, int, const TransferGeom&, int, const int*, hipStream_t);

template <typename T>
void launch_prolong(cplx<T>* out, const cplx<T>* in, const void* P, int pkind, const TransferGeom& g, int nrhs,
                    int accumulate, const int* flags, hipStream_t st) {
  if (blk_transfer(g)) {
    const dim3 grid((unsigned)((g.Vc * 2 + 3) / 4), 1);
#define AMG_PB(PT, RG) dispatch(prolong_blk_kernel<T, PT, 24, RG>, TrArgs<T, PT>{out, in, (const PT*)P, g, flags, accumulate, nrhs}, grid, dim3(256), st)
#define AMG_PB_RG(PT)                                                                    \
  if (nrhs == 1) { AMG_PB(PT, 1); } else if (nrhs <= 4) { AMG_PB(PT, 4); } else if (nrhs <= 8) { AMG_PB(PT, 8); } \
  else { AMG_PB(PT, 16); }
    if (pkind == P_F64) { AMG_PB_RG(double2) }
    else if (pkind == P_F32) { AMG_PB_RG(float2) }
    else { AMG_PB_RG(bf16x2) }
#undef AMG_PB_RG
#undef AMG_PB
    return;
  }
  dim3 grid(nblocks(g.Vf * g.dof), (unsigned)nrhs);
  if (pkind == P_F64)
    dispatch(prolong_kernel<T, double2>, TrArgs<T, double2>{out, in, (const double2*)P, g, flags, accumulate, nrhs}, grid, dim3(256), st);
  else if (pkind == P_F32)
    dispatch(prolong_kernel<T, float2>, TrArgs<T, float2>{out, in, (const float2*)P, g, flags, accumulate, nrhs}, grid, dim3(256), st);
  else
    dispatch(prolong_kernel<T, bf16x2>, TrArgs<T, bf16x2>{out, in, (const bf16x2*)P, g, flags, accumulate, nrhs}, grid, dim3(256), st);
}
template void launch_prolong<double>(double2*, const double2*, const void*, int, const TransferGeom&, int, int, const int*, hipStream_t);
template void launch_prolong<float>(float2*, const float2*, const void*, int, const TransferGeom&, int, int, const int*, hipStream_t);

void launch_orthonormalise(double2* P, const double2* vecs, const TransferGeom& g, int* err, hipStream_t st) {
  dim3 grid((unsigned)g.Vc, 2);
  const int dim = g.bs * (g.dof / 2);
  const int em = (dim + 63) / 64;
  if (em <= 1 || g.nv > 32 || em > 24) {
    hipLaunchKernelGGL(orthonormalise_kernel, grid, dim3(64), 0, st, P, vecs, g, err);
    return;
  }
#define AMG_ON(EM, NVM) hipLaunchKernelGGL((orthonormalise_cgs2_kernel<EM, NVM>), grid, dim3(64), 0, st, P, vecs, g, err)
#define AMG_ON_EM(EM)                          \
  if (g.nv <= 8) AMG_ON(EM, 8);                \
  else if (g.nv <= 16) AMG_ON(EM, 16);         \
  else if (g.nv <= 24) AMG_ON(EM, 24);         \
  else AMG_ON(EM, 32);
  if (em <= 2) { AMG_ON_EM(2) }
  else if (em <= 6) { AMG_ON_EM(6) }
  else if (em <= 12) { AMG_ON_EM(12) }
  else { AMG_ON_EM(24) }
#undef AMG_ON_EM
#undef AMG_ON
}

void launch_galerkin_scatter(double2* Y, const double2* R, long Vc, int nc, int nk, int t0, int chunk, hipStream_t st) {
  hipLaunchKernelGGL(galerkin_scatter_kernel, dim3(nblocks((long)nk * chunk * Vc * nc)), dim3(256), 0, st, Y, R, Vc,
                     nc, nk, t0, chunk);
}

void launch_unit_coarse(double2* E, long Vc, int nc, int t0, int chunk, hipStream_t st) {
  hipLaunchKernelGGL(unit_coarse_kernel, dim3(nblocks((long)chunk * Vc * nc)), dim3(256), 0, st, E, Vc, nc, t0, chunk);
}

}  // namespace amg

namespace amg {
namespace {
__global__ void diag_shift_kernel(double2* __restrict__ Y, const double2* __restrict__ M, long V, int nc, int ndir,
                                  double dm) {
  const long per = (long)nc * nc;
  const long total = V * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long site = i / per, e = i - site * per;
    double2 y = Y[site * ndir * per + e];
    const double2 m = M[i];
    y.x += dm * m.x; y.y += dm * m.y;
    Y[site * ndir * per + e] = y;
  }
}
}  // namespace

void launch_diag_shift(double2* Y, const double2* M, long V, int nc, int ndir, double dm, hipStream_t st) {
  long nb = (V * nc * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(diag_shift_kernel, dim3((unsigned)nb), dim3(256), 0, st, Y, M, V, nc, ndir, dm);
}
}  // namespace amg

namespace amg {
namespace {
__global__ void block_transpose_kernel(double2* __restrict__ out, const double2* __restrict__ in, long nblocks, int nc) {
  const long per = (long)nc * nc;
  const long total = nblocks * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long b = i / per;
    const long e = i - b * per;
    const int row = (int)(e / nc), col = (int)(e - (long)row * nc);
    out[i] = in[b * per + (long)col * nc + row];
  }
}
}  // namespace

void launch_block_transpose(double2* out, const double2* in, long nblocks, int nc, hipStream_t st) {
  long nb = (nblocks * nc * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(block_transpose_kernel, dim3((unsigned)nb), dim3(256), 0, st, out, in, nblocks, nc);
}

namespace {
// The stored prolongator as the dense rows of P at every fine site:
// out[fs][comp][t] (t = chi N_v + k) = P(fs)[comp][k] when comp has
// chirality chi, else 0; values of any storage kind widened to FP64.
template <typename PT>
__global__ void p_export_kernel(double2* __restrict__ out, const PT* __restrict__ P, TransferGeom g) {
  const int nc = 2 * g.nv, hd = g.dof / 2;
  const long total = g.Vf * g.dof * nc;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long fs = i / ((long)g.dof * nc);
    const int rem = (int)(i - fs * g.dof * nc);
    const int comp = rem / nc, t = rem - comp * nc;
    long j; int xi;
    BlockIdx::coarse_of(g, fs, j, xi);
    double2 v = make_double2(0.0, 0.0);
    if (comp / hd == t / g.nv) {
      const cplx<double> z = ldp<double>(gl(P), ((j * g.bs + xi) * g.dof + comp) * (long)g.nv + t % g.nv);
      v = z;
    }
    gl(out)[i] = v;
  }
}
}  // namespace

void launch_p_export(double2* out, const void* P, int pkind, const TransferGeom& g, hipStream_t st) {
  long nb = (g.Vf * g.dof * 2 * g.nv + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  if (pkind == P_F64)
    hipLaunchKernelGGL(p_export_kernel<double2>, dim3((unsigned)nb), dim3(256), 0, st, out, (const double2*)P, g);
  else if (pkind == P_F32)
    hipLaunchKernelGGL(p_export_kernel<float2>, dim3((unsigned)nb), dim3(256), 0, st, out, (const float2*)P, g);
  else
    hipLaunchKernelGGL(p_export_kernel<bf16x2>, dim3((unsigned)nb), dim3(256), 0, st, out, (const bf16x2*)P, g);
}
}  // namespace amg

// ---- right block-Jacobi preconditioning of a coarse level ------------------
// M(x) = A_0(x)^-1, the inverse of each site's diagonal block, and the
// operator A M of the preconditioned system: (A M)(x, x) = 1,
// (A M)(x, x + dir) = A_dir(x) M(x + dir).  GCR on A M y = b followed by
// x = M y gives the iterates of GCR on A x = b with the fixed preconditioner
// z = M r.  Blocks keep the stencil's column-major [col][row] order.
namespace amg {
namespace {
constexpr int BINV_MAX = 48;

// one wave per site: Gauss-Jordan with partial pivoting on [A_0 | 1] in LDS
// (nc <= BM: 32 KB for BM = 32, 72 KB for BM = 48, the 4d levels); err[0]
// is set when a pivot column is zero (the block is singular)
template <int BM>
__global__ __launch_bounds__(64) void block_inverse_kernel(double2* __restrict__ Minv, const double2* __restrict__ Y,
                                                           long V, int ndir, int nc, int* err) {
  __shared__ double2 a[BM][2 * BM];
  __shared__ double2 fac[BM];
  __shared__ int piv;
  const long site = blockIdx.x;
  if (site >= V) return;
  const int lane = threadIdx.x;
  const int w = 2 * nc;
  const double2* A0 = Y + site * ndir * (long)nc * nc;
  for (int e = lane; e < nc * w; e += 64) {
    const int r = e / w, c = e - r * w;
    a[r][c] = c < nc ? A0[(long)c * nc + r] : make_double2(c - nc == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int c = 0; c < nc; ++c) {
    {
      // pivot: the largest |a[r][c]| over r >= c (lowest r among equals),
      // a max-reduction over the lanes, one row each
      double m = -1.0;
      int p = nc;
      if (lane >= c && lane < nc) {
        m = a[lane][c].x * a[lane][c].x + a[lane][c].y * a[lane][c].y;
        p = lane;
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double mo = __shfl_xor(m, o, 64);
        const int po = __shfl_xor(p, o, 64);
        if (mo > m || (mo == m && po < p)) { m = mo; p = po; }
      }
      if (lane == 0) {
        if (!(m > 0.0)) {
          atomicOr(err, 1);
          p = -1;
        }
        piv = p;
      }
    }
    __syncthreads();
    const int p = piv;
    if (p < 0) return;  // uniform: the whole wave leaves
    if (p != c)
      for (int j = lane; j < w; j += 64) {
        const double2 t = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = t;
      }
    __syncthreads();
    const double2 d = a[c][c];
    const double dn = 1.0 / (d.x * d.x + d.y * d.y);
    const double2 inv = make_double2(d.x * dn, -d.y * dn);
    __syncthreads();
    for (int j = lane; j < w; j += 64) {
      const double2 v = a[c][j];
      a[c][j] = make_double2(v.x * inv.x - v.y * inv.y, v.x * inv.y + v.y * inv.x);
    }
    if (lane < nc && lane != c) fac[lane] = a[lane][c];
    __syncthreads();
    for (int e = lane; e < nc * w; e += 64) {
      const int r = e / w, j = e - r * w;
      if (r == c) continue;
      const double2 f = fac[r], u = a[c][j];
      double2 v = a[r][j];
      v.x -= f.x * u.x - f.y * u.y;
      v.y -= f.x * u.y + f.y * u.x;
      a[r][j] = v;
    }
    __syncthreads();
  }
  double2* M = Minv + site * (long)nc * nc;
  for (int e = lane; e < nc * nc; e += 64) {
    const int col = e / nc, row = e - col * nc;
    M[e] = a[row][nc + col];
  }
}

// thread per entry (site, k, col, row) of A M
__global__ __launch_bounds__(256) void jacobi_couplings_kernel(double2* __restrict__ AM, const double2* __restrict__ Y,
                                                               const double2* __restrict__ Minv, CoarseGeom g) {
  const int nc = g.nc, nd = g.nd, ndir = 2 * nd + 1;
  const long per = (long)nc * nc;
  const long total = g.V * ndir * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long site = i / (ndir * per);
    const long rem = i - site * ndir * per;
    const int k = (int)(rem / per);
    const int col = (int)((rem - (long)k * per) / nc), row = (int)(rem - (long)k * per - (long)col * nc);
    if (k == 0) {
      AM[i] = make_double2(col == row ? 1.0 : 0.0, 0.0);
      continue;
    }
    int x[4];
    coords(site, g.dims, nd, x);
    const long nb = neighbour(site, x, g.dims, nd, k - 1);
    const double2* Ak = Y + (site * ndir + k) * per;  // [m][row]
    const double2* Mn = Minv + nb * per + (long)col * nc;  // column col of M(nb): [m]
    double sr = 0.0, si = 0.0;
    for (int m = 0; m < nc; ++m) {
      const double2 u = Ak[(long)m * nc + row], v = Mn[m];
      sr += u.x * v.x - u.y * v.y;
      si += u.x * v.y + u.y * v.x;
    }
    AM[i] = make_double2(sr, si);
  }
}

// out(x) = M(x) in(x) for every site and right-hand side (grid y = rhs)
template <typename T>
__global__ __launch_bounds__(256) void block_apply_kernel(cplx<T>* __restrict__ out, const cplx<T>* __restrict__ in,
                                                          const cplx<T>* __restrict__ M, long V, int nc) {
  const long n = V * nc;
  const long ro = (long)blockIdx.y * n;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long site = i / nc;
    const int row = (int)(i - site * nc);
    const cplx<T>* Ms = M + site * (long)nc * nc + row;
    const cplx<T>* v = in + ro + site * nc;
    T sr = 0, si = 0;
    for (int col = 0; col < nc; ++col) {
      const cplx<T> u = Ms[(long)col * nc], w = v[col];
      sr += u.x * w.x - u.y * w.y;
      si += u.x * w.y + u.y * w.x;
    }
    out[ro + i] = mk<T>(sr, si);
  }
}
}  // namespace

bool block_jacobi_supported(int nc) { return nc >= 1 && nc <= BINV_MAX; }

void launch_block_inverse(double2* Minv, const double2* Y, long V, int ndir, int nc, int* err, hipStream_t st) {
  if (nc <= 32)
    hipLaunchKernelGGL(block_inverse_kernel<32>, dim3((unsigned)V), dim3(64), 0, st, Minv, Y, V, ndir, nc, err);
  else
    hipLaunchKernelGGL(block_inverse_kernel<48>, dim3((unsigned)V), dim3(64), 0, st, Minv, Y, V, ndir, nc, err);
}

void launch_jacobi_couplings(double2* AM, const double2* Y, const double2* Minv, const CoarseGeom& g, hipStream_t st) {
  long nb = (g.V * (2 * g.nd + 1) * (long)g.nc * g.nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(jacobi_couplings_kernel, dim3((unsigned)nb), dim3(256), 0, st, AM, Y, Minv, g);
}

template <typename T>
void launch_block_apply(cplx<T>* out, const cplx<T>* in, const cplx<T>* M, long V, int nc, int nrhs, hipStream_t st) {
  long nb = (V * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(block_apply_kernel<T>, dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, st, out, in, M, V, nc);
}
template void launch_block_apply<double>(double2*, const double2*, const double2*, long, int, int, hipStream_t);
template void launch_block_apply<float>(float2*, const float2*, const float2*, long, int, int, hipStream_t);
}  // namespace amg

// ---- even-odd reduction of the block-Jacobi preconditioned coarsest level --
// 2d coarse lattices with even extents.  With T = A M (unit diagonal) split
// by site parity, T y = b becomes (1 - T_eo T_oe) y_e = b_e - T_eo b_o and
// y_o = b_o - T_oe y_e.  Half-lattice fields hold the sites of one parity
// in site order: half index h = s / 2.  Coupling blocks of one parity:
// C[h][dir][col][row], the coupling of site s(h) to its neighbour in
// direction dir (dir = 2 mu: +mu, 2 mu + 1: -mu).
namespace amg {
namespace {
__device__ __forceinline__ long eo_site(long h, int L1, int par) {
  const long y = h / (L1 / 2);
  const long x = 2 * (h - y * (L1 / 2)) + ((y + par) & 1);
  return x + y * L1;
}

__global__ __launch_bounds__(256) void eo_split_kernel(double2* __restrict__ Ce, double2* __restrict__ Co,
                                                       const double2* __restrict__ T, int L1, int L2, int nc) {
  const long per = (long)nc * nc;
  const long Vh = (long)L1 * L2 / 2;
  const long total = 2 * Vh * 4 * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int par = (int)(i / (Vh * 4 * per));
    const long rem = i - (long)par * Vh * 4 * per;
    const long h = rem / (4 * per);
    const long e = rem - h * 4 * per;  // dir * per + col * nc + row
    const int dir = (int)(e / per);
    const long s = eo_site(h, L1, par);
    (par ? Co : Ce)[rem] = T[(s * 5 + 1 + dir) * per + (e - (long)dir * per)];
  }
}

// out(h) = sum_dir C[h][dir] in(nb_dir(s(h)))           (EPI 0)
//        = b(h) - sum_dir C[h][dir] in(...)            (EPI 1)
//        = b(h) - b2(h) + sum_dir C[h][dir] in(...)    (EPI 2)
// for the sites of parity `par`; in, b are half fields (of the other / this
// parity) or full fields when in_full / b_full.  Thread per (site, row).
template <typename T>
struct EoArgs {
  cplx<T>* out;
  const cplx<T>* in;
  const cplx<T>* b;
  const cplx<T>* b2;
  const cplx<T>* C;
  int L1, L2, nc, par, in_full, b_full;
  int nrhs;
  cplx<T>* out2;  // optional second copy of out
  cplx<T>* zero;  // optional half field set to zero
};
// NCM > 0: nc <= NCM; four adjacent lanes take the four directions of one
// row, each issuing all loads of its direction at once (clamped column,
// surplus terms skipped), and add their sums with two lane exchanges.
// NCM = 0: any nc up to 32, one thread per row, one column at a time.
template <typename T, int EPI, int NCM>
__global__ __launch_bounds__(256) void eo_hop_kernel(EoArgs<T> a0, const EoArgs<T>* batch) {
  AMG_ARGS(EoArgs<T>)
  const int L1 = a.L1, L2 = a.L2, nc = a.nc;
  const long Vh = (long)L1 * L2 / 2;
  const long n = Vh * nc;
  const int rhs = blockIdx.y;
  const long oh = (long)rhs * n, of = 2 * oh;
  const cplx<T>* pin = a.in + (a.in_full ? of : oh);
  constexpr int LPR = NCM > 0 ? 4 : 1;  // lanes per row
  // the stride is a multiple of 64, so the lanes of a row stay in one wave
  for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < n * LPR; j += (long)gridDim.x * blockDim.x) {
    const long i = j / LPR;
    const int dl = (int)(j - i * LPR);
    const long h = i / nc;
    const int row = (int)(i - h * nc);
    const long s = eo_site(h, L1, a.par);
    const int x = (int)(s % L1), y = (int)(s / L1);
    long nb[4];
    nb[0] = (x == L1 - 1) ? s - (L1 - 1) : s + 1;
    nb[1] = (x == 0) ? s + (L1 - 1) : s - 1;
    nb[2] = (y == L2 - 1) ? s - (long)(L2 - 1) * L1 : s + L1;
    nb[3] = (y == 0) ? s + (long)(L2 - 1) * L1 : s - L1;
    T sr = 0, si = 0;
    if (NCM > 0) {
      const long nbd = dl == 0 ? nb[0] : dl == 1 ? nb[1] : dl == 2 ? nb[2] : nb[3];
      const cplx<T>* Cd = a.C + (h * 4 + dl) * (long)nc * nc + row;
      const cplx<T>* v = pin + (a.in_full ? nbd : nbd >> 1) * nc;
      cplx<T> cu[NCM > 0 ? NCM : 1], cw[NCM > 0 ? NCM : 1];
#pragma unroll
      for (int col = 0; col < NCM; ++col) {
        const int c = col < nc ? col : nc - 1;
        cu[col] = Cd[(long)c * nc];
        cw[col] = v[c];
      }
#pragma unroll
      for (int col = 0; col < NCM; ++col) {
        if (col < nc) {
          sr += cu[col].x * cw[col].x - cu[col].y * cw[col].y;
          si += cu[col].x * cw[col].y + cu[col].y * cw[col].x;
        }
      }
      sr += __shfl_xor(sr, 1, 64);
      si += __shfl_xor(si, 1, 64);
      sr += __shfl_xor(sr, 2, 64);
      si += __shfl_xor(si, 2, 64);
      if (dl != 0) continue;
    } else {
      for (int d = 0; d < 4; ++d) {
        const cplx<T>* Cd = a.C + (h * 4 + d) * (long)nc * nc + row;
        const cplx<T>* v = pin + (a.in_full ? nb[d] : nb[d] >> 1) * nc;
        for (int col = 0; col < nc; ++col) {
          const cplx<T> u = Cd[(long)col * nc], w = v[col];
          sr += u.x * w.x - u.y * w.y;
          si += u.x * w.y + u.y * w.x;
        }
      }
    }
    cplx<T> v = mk<T>(sr, si);
    if (EPI >= 1) {
      const cplx<T> bv = a.b[a.b_full ? of + s * nc + row : oh + i];
      if (EPI == 1) {
        v = mk<T>(bv.x - sr, bv.y - si);
      } else {
        const cplx<T> b2v = a.b2[oh + i];
        v = mk<T>(bv.x - b2v.x + sr, bv.y - b2v.y + si);
      }
    }
    a.out[oh + i] = v;
    if (a.out2) a.out2[oh + i] = v;
    if (a.zero) a.zero[oh + i] = mk<T>(0, 0);
  }
}

// The same for N_c = 16 with one wave per site in the lane layout of
// coarse16_kernel (C16): the loads of all four directions are issued before
// the first multiply-add, then the partial row sums are reduced across the
// lanes that share the rows.
template <typename T, int EPI>
__global__ __launch_bounds__(256) void eo16_kernel(EoArgs<T> a0, const EoArgs<T>* batch) {
  AMG_ARGS(EoArgs<T>)
  using K = C16<T>;
  const int L1 = a.L1, L2 = a.L2;
  const long Vh = (long)L1 * L2 / 2;
  const int rhs = blockIdx.y;
  const long oh = (long)rhs * Vh * K::NC, of = 2 * oh;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + (a.in_full ? of : oh);
  gptr<const cplx<T>> __restrict__ C = gl(a.C);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = lane / K::LPC, rg = lane - cg * K::LPC;
  for (long h = (long)blockIdx.x * 4 + wave; h < Vh; h += (long)gridDim.x * 4) {
    const long s = eo_site(h, L1, a.par);
    const int x = (int)(s % L1), y = (int)(s / L1);
    long nb[4];
    nb[0] = (x == L1 - 1) ? s - (L1 - 1) : s + 1;
    nb[1] = (x == 0) ? s + (L1 - 1) : s - 1;
    nb[2] = (y == L2 - 1) ? s - (long)(L2 - 1) * L1 : s + L1;
    nb[3] = (y == 0) ? s + (long)(L2 - 1) * L1 : s - L1;
    // this lane's rows of b and b2 (lanes of column group 0 write the result)
    cplx<T> bv[K::R], b2v[K::R];
#pragma unroll
    for (int i = 0; i < K::R; ++i) {
      const int row = rg * K::R + i;
      bv[i] = mk<T>(0, 0);
      b2v[i] = mk<T>(0, 0);
      if (cg == 0 && EPI >= 1) bv[i] = a.b[a.b_full ? of + s * K::NC + row : oh + h * K::NC + row];
      if (cg == 0 && EPI == 2) b2v[i] = a.b2[oh + h * K::NC + row];
    }
    gptr<const cplx<T>> __restrict__ Cs = C + h * 4L * K::NC * K::NC + rg * K::R;
    cplx<T> ev[4][K::NQ], yv[4][K::NQ][K::R];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        ev[d][q] = pin[(a.in_full ? nb[d] : nb[d] >> 1) * K::NC + col];
#pragma unroll
        for (int i = 0; i < K::R; ++i) yv[d][q][i] = Cs[(long)d * K::NC * K::NC + col * K::NC + i];
      }
    cplx<T> acc[K::R];
#pragma unroll
    for (int i = 0; i < K::R; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q)
#pragma unroll
        for (int i = 0; i < K::R; ++i) cfma<T>(acc[i], yv[d][q][i], ev[d][q]);
#pragma unroll
    for (int i = 0; i < K::R; ++i) {
#pragma unroll
      for (int o = K::LPC; o < 64; o <<= 1) {
        acc[i].x += __shfl_xor(acc[i].x, o, 64);
        acc[i].y += __shfl_xor(acc[i].y, o, 64);
      }
    }
    if (cg == 0) {
#pragma unroll
      for (int i = 0; i < K::R; ++i) {
        const int row = rg * K::R + i;
        cplx<T> v = acc[i];
        if (EPI == 1) v = mk<T>(bv[i].x - v.x, bv[i].y - v.y);
        if (EPI == 2) v = mk<T>(bv[i].x - b2v[i].x + v.x, bv[i].y - b2v[i].y + v.y);
        a.out[oh + h * K::NC + row] = v;
        if (a.out2) a.out2[oh + h * K::NC + row] = v;
        if (a.zero) a.zero[oh + h * K::NC + row] = mk<T>(0, 0);
      }
    }
  }
}

// The reduced operator 1 - T_eo T_oe as a stencil on the even sites: the
// two-hop paths from an even site end on the site itself, at (+-2, 0),
// (0, +-2) or (+-1, +-1).  Offsets k = 0: (0, 0), 1: (2, 0), 2: (-2, 0),
// 3: (0, 2), 4: (0, -2), 5: (1, 1), 6: (1, -1), 7: (-1, 1), 8: (-1, -1);
// S_k(x) = [k = 0] 1 - sum over the paths (d1, d2) of offset k of
// T_eo(x, d1) T_oe(x + d1, d2), directions d = 0: +x, 1: -x, 2: +y, 3: -y.
// Blocks [h][k][col][row] (FP64), thread per entry.
__constant__ int kS9Paths[9][4][2] = {
    {{0, 1}, {1, 0}, {2, 3}, {3, 2}}, {{0, 0}, {-1, -1}, {-1, -1}, {-1, -1}}, {{1, 1}, {-1, -1}, {-1, -1}, {-1, -1}},
    {{2, 2}, {-1, -1}, {-1, -1}, {-1, -1}}, {{3, 3}, {-1, -1}, {-1, -1}, {-1, -1}}, {{0, 2}, {2, 0}, {-1, -1}, {-1, -1}},
    {{0, 3}, {3, 0}, {-1, -1}, {-1, -1}}, {{1, 2}, {2, 1}, {-1, -1}, {-1, -1}}, {{1, 3}, {3, 1}, {-1, -1}, {-1, -1}}};

__device__ __forceinline__ long nb2d(long s, int L1, int L2, int d) {
  const int x = (int)(s % L1), y = (int)(s / L1);
  if (d == 0) return (x == L1 - 1) ? s - (L1 - 1) : s + 1;
  if (d == 1) return (x == 0) ? s + (L1 - 1) : s - 1;
  if (d == 2) return (y == L2 - 1) ? s - (long)(L2 - 1) * L1 : s + L1;
  return (y == 0) ? s + (long)(L2 - 1) * L1 : s - L1;
}

__global__ __launch_bounds__(256) void eo_schur_build_kernel(double2* __restrict__ S9, const double2* __restrict__ Ce,
                                                             const double2* __restrict__ Co, int L1, int L2, int nc) {
  const long per = (long)nc * nc;
  const long Vh = (long)L1 * L2 / 2;
  const long total = Vh * 9 * per;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const long h = i / (9 * per);
    const long rem = i - h * 9 * per;
    const int k = (int)(rem / per);
    const int col = (int)((rem - (long)k * per) / nc), row = (int)(rem - (long)k * per - (long)col * nc);
    const long s = eo_site(h, L1, 0);
    double sr = (k == 0 && row == col) ? 1.0 : 0.0, si = 0.0;
    for (int p = 0; p < 4; ++p) {
      const int d1 = kS9Paths[k][p][0], d2 = kS9Paths[k][p][1];
      if (d1 < 0) break;
      const long ho = nb2d(s, L1, L2, d1) >> 1;  // the odd site between
      const double2* A = Ce + (h * 4 + d1) * per;    // [m][row]
      const double2* B = Co + (ho * 4 + d2) * per;   // [col][m]
      for (int m = 0; m < nc; ++m) {
        const double2 u = A[(long)m * nc + row], v = B[(long)col * nc + m];
        sr -= u.x * v.x - u.y * v.y;
        si -= u.x * v.y + u.y * v.x;
      }
    }
    S9[i] = make_double2(sr, si);
  }
}

// out(h) = sum_k S_k(h) in(h + offset_k)            (EPI 0)
//        = b(h) - sum_k S_k(h) in(h + offset_k)     (EPI 1)
// on the even half field, N_c = 16, one wave per site (C16 lane layout).
template <typename T, int EPI>
__global__ __launch_bounds__(256) void eo_s9_kernel(EoArgs<T> a0, const EoArgs<T>* batch) {
  AMG_ARGS(EoArgs<T>)
  using K = C16<T>;
  const int L1 = a.L1, L2 = a.L2;
  const long Vh = (long)L1 * L2 / 2;
  const int rhs = blockIdx.y;
  const long oh = (long)rhs * Vh * K::NC;
  gptr<const cplx<T>> __restrict__ pin = gl(a.in) + oh;
  gptr<const cplx<T>> __restrict__ C = gl(a.C);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cg = lane / K::LPC, rg = lane - cg * K::LPC;
  for (long h = (long)blockIdx.x * 4 + wave; h < Vh; h += (long)gridDim.x * 4) {
    const long s = eo_site(h, L1, 0);
    const int x = (int)(s % L1), y = (int)(s / L1);
    const int xp = x + 1 == L1 ? 0 : x + 1, xm = x == 0 ? L1 - 1 : x - 1;
    const int yp = y + 1 == L2 ? 0 : y + 1, ym = y == 0 ? L2 - 1 : y - 1;
    const int xpp = xp + 1 == L1 ? 0 : xp + 1, xmm = xm == 0 ? L1 - 1 : xm - 1;
    const int ypp = yp + 1 == L2 ? 0 : yp + 1, ymm = ym == 0 ? L2 - 1 : ym - 1;
    long nb[9];
    nb[0] = s;
    nb[1] = xpp + (long)y * L1;
    nb[2] = xmm + (long)y * L1;
    nb[3] = x + (long)ypp * L1;
    nb[4] = x + (long)ymm * L1;
    nb[5] = xp + (long)yp * L1;
    nb[6] = xp + (long)ym * L1;
    nb[7] = xm + (long)yp * L1;
    nb[8] = xm + (long)ym * L1;
    cplx<T> bv[K::R];
#pragma unroll
    for (int i = 0; i < K::R; ++i) {
      bv[i] = mk<T>(0, 0);
      if (cg == 0 && EPI == 1) bv[i] = a.b[oh + h * K::NC + rg * K::R + i];
    }
    gptr<const cplx<T>> __restrict__ Cs = C + h * 9L * K::NC * K::NC + rg * K::R;
    cplx<T> ev[9][K::NQ], yv[9][K::NQ][K::R];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q) {
        const int col = cg + K::CPI * q;
        ev[k][q] = pin[(nb[k] >> 1) * K::NC + col];
#pragma unroll
        for (int i = 0; i < K::R; ++i) yv[k][q][i] = Cs[(long)k * K::NC * K::NC + col * K::NC + i];
      }
    cplx<T> acc[K::R];
#pragma unroll
    for (int i = 0; i < K::R; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int q = 0; q < K::NQ; ++q)
#pragma unroll
        for (int i = 0; i < K::R; ++i) cfma<T>(acc[i], yv[k][q][i], ev[k][q]);
#pragma unroll
    for (int i = 0; i < K::R; ++i) {
#pragma unroll
      for (int o = K::LPC; o < 64; o <<= 1) {
        acc[i].x += __shfl_xor(acc[i].x, o, 64);
        acc[i].y += __shfl_xor(acc[i].y, o, 64);
      }
    }
    if (cg == 0) {
#pragma unroll
      for (int i = 0; i < K::R; ++i) {
        cplx<T> v = acc[i];
        if (EPI == 1) v = mk<T>(bv[i].x - v.x, bv[i].y - v.y);
        a.out[oh + h * K::NC + rg * K::R + i] = v;
      }
    }
  }
}

// x(s) = M(s) y(s) with y split into its even and odd half fields
// (NCM > 0: nc <= NCM, all loads of a row issued at once)
template <typename T, int NCM>
__global__ __launch_bounds__(256) void eo_block_apply_kernel(cplx<T>* __restrict__ x, const cplx<T>* __restrict__ ye,
                                                             const cplx<T>* __restrict__ yo, const cplx<T>* __restrict__ M,
                                                             int L1, int L2, int nc) {
  const long V = (long)L1 * L2;
  const long n = V * nc;
  const int rhs = blockIdx.y;
  const long of = (long)rhs * n, oh = of / 2;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long s = i / nc;
    const int row = (int)(i - s * nc);
    const int par = (int)(((s % L1) + s / L1) & 1);
    const cplx<T>* v = (par ? yo : ye) + oh + (s >> 1) * nc;
    const cplx<T>* Ms = M + s * (long)nc * nc + row;
    T sr = 0, si = 0;
    if (NCM > 0) {
      cplx<T> cu[NCM > 0 ? NCM : 1], cw[NCM > 0 ? NCM : 1];
#pragma unroll
      for (int col = 0; col < NCM; ++col) {
        const int c = col < nc ? col : nc - 1;
        cu[col] = Ms[(long)c * nc];
        cw[col] = v[c];
      }
#pragma unroll
      for (int col = 0; col < NCM; ++col) {
        if (col < nc) {
          sr += cu[col].x * cw[col].x - cu[col].y * cw[col].y;
          si += cu[col].x * cw[col].y + cu[col].y * cw[col].x;
        }
      }
    } else {
      for (int col = 0; col < nc; ++col) {
        const cplx<T> u = Ms[(long)col * nc], w = v[col];
        sr += u.x * w.x - u.y * w.y;
        si += u.x * w.y + u.y * w.x;
      }
    }
    x[of + i] = mk<T>(sr, si);
  }
}
}  // namespace

bool eo_supported(int nd, const int* dims, int nc) {
  return nd == 2 && dims[0] % 2 == 0 && dims[1] % 2 == 0 && dims[0] >= 2 && dims[1] >= 2 && nc >= 1 && nc <= 32;
}

void launch_eo_split(double2* Ce, double2* Co, const double2* T, int L1, int L2, int nc, hipStream_t st) {
  long nb = ((long)L1 * L2 * 4 * nc * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(eo_split_kernel, dim3((unsigned)nb), dim3(256), 0, st, Ce, Co, T, L1, L2, nc);
}

template <typename T>
void launch_eo_hop(cplx<T>* out, const cplx<T>* in, const cplx<T>* b, const cplx<T>* b2, const cplx<T>* C, int L1,
                   int L2, int nc, int par, int in_full, int b_full, int epi, int nrhs, hipStream_t st, cplx<T>* out2,
                   cplx<T>* zero) {
  long nb = ((long)L1 * L2 / 2 * nc * (nc <= 16 ? 4 : 1) + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  const dim3 g((unsigned)nb, (unsigned)nrhs);
  EoArgs<T> a{out, in, b, b2, C, L1, L2, nc, par, in_full, b_full, nrhs, out2, zero};
  if (nc == 16) {
    const long Vh = (long)L1 * L2 / 2;
    long nw = (Vh + 3) / 4;
    if (nw > (1L << 20)) nw = 1L << 20;
    const dim3 g16((unsigned)nw, (unsigned)nrhs);
    if (epi == 0) dispatch(eo16_kernel<T, 0>, a, g16, dim3(256), st);
    else if (epi == 1) dispatch(eo16_kernel<T, 1>, a, g16, dim3(256), st);
    else dispatch(eo16_kernel<T, 2>, a, g16, dim3(256), st);
    return;
  }
#define AMG_EOH(NCM)                                                         \
  {                                                                          \
    if (epi == 0) dispatch(eo_hop_kernel<T, 0, NCM>, a, g, dim3(256), st);   \
    else if (epi == 1) dispatch(eo_hop_kernel<T, 1, NCM>, a, g, dim3(256), st); \
    else dispatch(eo_hop_kernel<T, 2, NCM>, a, g, dim3(256), st);            \
    return;                                                                  \
  }
  if (nc <= 4) AMG_EOH(4)
  if (nc <= 8) AMG_EOH(8)
  if (nc <= 16) AMG_EOH(16)
#undef AMG_EOH
  if (epi == 0) dispatch(eo_hop_kernel<T, 0, 0>, a, g, dim3(256), st);
  else if (epi == 1) dispatch(eo_hop_kernel<T, 1, 0>, a, g, dim3(256), st);
  else dispatch(eo_hop_kernel<T, 2, 0>, a, g, dim3(256), st);
}
template void launch_eo_hop<double>(double2*, const double2*, const double2*, const double2*, const double2*, int, int,
                                    int, int, int, int, int, int, hipStream_t, double2*, double2*);
template void launch_eo_hop<float>(float2*, const float2*, const float2*, const float2*, const float2*, int, int, int,
                                   int, int, int, int, int, hipStream_t, float2*, float2*);

void launch_eo_schur_build(double2* S9, const double2* Ce, const double2* Co, int L1, int L2, int nc, hipStream_t st) {
  long nb = ((long)L1 * L2 / 2 * 9 * nc * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  hipLaunchKernelGGL(eo_schur_build_kernel, dim3((unsigned)nb), dim3(256), 0, st, S9, Ce, Co, L1, L2, nc);
}

template <typename T>
void launch_eo_s9(cplx<T>* out, const cplx<T>* in, const cplx<T>* b, const cplx<T>* S9, int L1, int L2, int epi,
                  int nrhs, hipStream_t st) {
  const long Vh = (long)L1 * L2 / 2;
  long nw = (Vh + 3) / 4;
  if (nw > (1L << 20)) nw = 1L << 20;
  const dim3 g((unsigned)nw, (unsigned)nrhs);
  EoArgs<T> a{out, in, b, nullptr, S9, L1, L2, 16, 0, 0, 0, nrhs, nullptr, nullptr};
  if (epi == 0) dispatch(eo_s9_kernel<T, 0>, a, g, dim3(256), st);
  else dispatch(eo_s9_kernel<T, 1>, a, g, dim3(256), st);
}
template void launch_eo_s9<double>(double2*, const double2*, const double2*, const double2*, int, int, int, int,
                                   hipStream_t);
template void launch_eo_s9<float>(float2*, const float2*, const float2*, const float2*, int, int, int, int,
                                  hipStream_t);

template <typename T>
void launch_eo_block_apply(cplx<T>* x, const cplx<T>* ye, const cplx<T>* yo, const cplx<T>* M, int L1, int L2, int nc,
                           int nrhs, hipStream_t st) {
  long nb = ((long)L1 * L2 * nc + 255) / 256;
  if (nb > (1L << 20)) nb = 1L << 20;
  if (nc <= 16)
    hipLaunchKernelGGL((eo_block_apply_kernel<T, 16>), dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, st, x, ye, yo,
                       M, L1, L2, nc);
  else
    hipLaunchKernelGGL((eo_block_apply_kernel<T, 0>), dim3((unsigned)nb, (unsigned)nrhs), dim3(256), 0, st, x, ye, yo,
                       M, L1, L2, nc);
}
template void launch_eo_block_apply<double>(double2*, const double2*, const double2*, const double2*, int, int, int, int,
                                            hipStream_t);
template void launch_eo_block_apply<float>(float2*, const float2*, const float2*, const float2*, int, int, int, int,
                                           hipStream_t);
}  // namespace amg

// Coarse block stencil for many right-hand sides at once, on the matrix cores.
//
// out[r][x] = sum_k Y_k(x) in[r][x + d_k]  (k = 0 the diagonal block, then
// +mu / -mu), the coarse operator of Eq. (2) in the layout of the other
// coarse kernels: fields [rhs][site][t], blocks Y[site][k][col][row].
//
// Per site and direction this is a complex (NC x NC) x (NC x R) product.
// With R right-hand sides in flight every block of Y is read from HBM once
// instead of R times, which is what makes the multi-rhs coarse apply dense
// enough for MFMA: the complex product is split into four real products
// (Re Y Re X - Im Y Im X, Re Y Im X + Im Y Re X) accumulated by
// v_mfma_f32_16x16x4_f32 in 16-row tiles (one wave per tile) and 4-column
// steps.  The neighbour's input block, [rhs][NC] in memory, is staged in LDS
// as [NC][rhs] so that the B operand of a step (4 columns x 16 rhs) is one
// conflict-free LDS read.  Right-hand sides go in groups of 16 (the MFMA N
// dimension); an unused column of a group is zero.
//
// Operand layouts of v_mfma_f32_16x16x4_f32 (64 lanes): A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[4 q + e][j] in element e of lane
// j + 16 q.
#include <hip/hip_runtime.h>

#include "common.h"
#include "dispatch.h"
#include "kernels.h"

namespace amg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ long mr_neighbour(long site, const CoarseGeom& g, int dir) {
  // dir = 2 mu (+mu) or 2 mu + 1 (-mu), periodic
  const int mu = dir >> 1;
  long stride = 1;
#pragma unroll
  for (int nu = 0; nu < 3; ++nu)
    if (nu < mu) stride *= g.dims[nu];
  const int L = at4(g.dims, mu);
  const int x = (int)((site / stride) % L);
  if ((dir & 1) == 0) return (x == L - 1) ? site - (long)(L - 1) * stride : site + stride;
  return (x == 0) ? site + (long)(L - 1) * stride : site - stride;
}

constexpr int RG = 16;  // right-hand sides per group (MFMA N)

template <int NC, int DAG, int EPI>
__global__ __launch_bounds__(NC / 16 * 64) void coarse_mrhs_kernel(CoarseArgs<float> a0,
                                                                    const CoarseArgs<float>* batch) {
  AMG_ARGS(CoarseArgs<float>)
  constexpr int NT = NC / 16;       // row tiles = waves per block
  constexpr int NTHR = NT * 64;
  __shared__ float2 xs[NC][RG + 1];  // +1: stride 136 B spreads the staging stores over the banks
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ndir = 2 * a.g.nd + 1;
  const long V = a.g.V;
  const long rstride = V * NC;
  const int row = wave * 16 + (lane & 15);   // A operand row of this lane
  const int kq = lane >> 4;                  // k within a 4-column step
  for (long site = blockIdx.x; site < V; site += gridDim.x) {
    for (int r0 = 0; r0 < a.nrhs; r0 += RG) {
      f32x4 accr = {0.f, 0.f, 0.f, 0.f}, acci = {0.f, 0.f, 0.f, 0.f};
      for (int k = 0; k < ndir; ++k) {
        const long nb = (k == 0) ? site : mr_neighbour(site, a.g, k - 1);
        __syncthreads();  // the previous direction's reads of xs are done
        for (int e = threadIdx.x; e < RG * NC; e += NTHR) {
          const int rr = e / NC, col = e - rr * NC;
          const int rhs = r0 + rr;
          float2 v = make_float2(0.f, 0.f);
          if (rhs < a.nrhs && !skip_rhs(a.red.flags, rhs)) {
            v = gl(a.in)[rhs * rstride + nb * NC + col];
            if (DAG && col >= NC / 2) v = make_float2(-v.x, -v.y);
          }
          xs[col][rr] = v;
        }
        __syncthreads();
        gptr<const float2> __restrict__ Yk = gl(a.Y) + ((site * ndir + k) * NC) * (long)NC;
        float2 y[NC / 4];
#pragma unroll
        for (int s = 0; s < NC / 4; ++s) y[s] = Yk[(long)(4 * s + kq) * NC + row];
#pragma unroll
        for (int s = 0; s < NC / 4; ++s) {
          const float2 x = xs[4 * s + kq][lane & 15];
          accr = __builtin_amdgcn_mfma_f32_16x16x4f32(y[s].x, x.x, accr, 0, 0, 0);
          accr = __builtin_amdgcn_mfma_f32_16x16x4f32(-y[s].y, x.y, accr, 0, 0, 0);
          acci = __builtin_amdgcn_mfma_f32_16x16x4f32(y[s].x, x.y, acci, 0, 0, 0);
          acci = __builtin_amdgcn_mfma_f32_16x16x4f32(y[s].y, x.x, acci, 0, 0, 0);
        }
      }
      const int rhs = r0 + (lane & 15);
      if (rhs < a.nrhs && !skip_rhs(a.red.flags, rhs)) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int orow = wave * 16 + 4 * kq + e;
          float2 v = make_float2(accr[e], acci[e]);
          if (DAG && orow >= NC / 2) v = make_float2(-v.x, -v.y);
          const long idx = rhs * rstride + site * NC + orow;
          if (EPI == EPI_RESID) {
            const float2 bv = gl(a.b)[idx];
            v = make_float2(bv.x - v.x, bv.y - v.y);
          }
          gl(a.out)[idx] = v;
        }
      }
    }
    if (a.copy_out) {
      for (int e = threadIdx.x; e < a.nrhs * NC; e += NTHR) {
        const int rhs = e / NC, col = e - rhs * NC;
        if (skip_rhs(a.red.flags, rhs)) continue;
        const long idx = rhs * rstride + site * NC + col;
        gl(a.copy_out)[idx] = gl(a.in)[idx];
      }
    }
  }
}

}  // namespace

bool coarse_mrhs_supported(int nc, int epi) { return (nc == 16 || nc == 48) && (epi == EPI_PLAIN || epi == EPI_RESID); }

void launch_coarse_mrhs(const CoarseArgs<float>& a, int dagger, int epi, hipStream_t st) {
  long nb = a.g.V;
  if (nb > 65536) nb = 65536;
  const dim3 grid((unsigned)nb, 1);
#define AMG_MR(NC, DAG, EPI) dispatch(coarse_mrhs_kernel<NC, DAG, EPI>, a, grid, dim3(NC / 16 * 64), st)
#define AMG_MR_NC(NC)                                  \
  if (epi == EPI_RESID) {                              \
    if (dagger) { AMG_MR(NC, 1, EPI_RESID); } else { AMG_MR(NC, 0, EPI_RESID); } \
  } else {                                             \
    if (dagger) { AMG_MR(NC, 1, EPI_PLAIN); } else { AMG_MR(NC, 0, EPI_PLAIN); } \
  }
  if (a.g.nc == 48) {
    AMG_MR_NC(48)
  } else {
    AMG_MR_NC(16)
  }
#undef AMG_MR_NC
#undef AMG_MR
}

}  // namespace amg

// Learned setup: a small local convolutional network that proposes initial
// near-null vectors for the adaptive setup (2d U(1)), with its own training
// kernels on gfx950.
//
// Network: four 3x3 convolutions with periodic padding, channels
// 4 -> 64 -> 64 -> 64 -> 32, tanh between layers.  Input per site:
// cos/sin of the two link angles after block-local tree gauge fixing (links
// of a maximal tree inside every 4x4 block set to 1), which makes the block
// span of the near-null vectors a gauge-invariant target.  Output per site:
// 8 complex vectors x 2 spin components (channel 4k + 2s + re/im), mapped
// back by the inverse gauge transformation.
//
// Storage: activations and the compute copy of the weights in bfloat16 (or
// FP32), gradients and accumulation in FP32, master weights FP32 (Adam).
// Loss: for each 4x4 block and chirality s (= spin), with V the 16 x 8
// block-restricted predictions and t_k the normalised targets,
// L = sum_k (1 - u_k^dag A u_k), u_k = V^dag t_k, A = (V^dag V + eps)^-1,
// and dL/d(conj V) = -sum_k t_k w_k^dag + V sum_k w_k w_k^dag, w_k = A u_k,
// evaluated in FP64 per (block, chirality).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "amg.h"
#include "common.h"
#include "hostutil.h"

using namespace amg;
using namespace amg::host;

namespace {

constexpr int NL = 4;
constexpr int CH[NL + 1] = {4, 64, 64, 64, 32};
constexpr int NVEC = 8;
constexpr int BLK = 4;          // gauge-fixing / loss block extent
constexpr double LOSS_EPS = 1e-3;

struct bf16s { uint16_t v; };
__device__ __forceinline__ float ld(const float* p, long i) { return p[i]; }
__device__ __forceinline__ float ld(const bf16s* p, long i) { return bf2f(p[i].v); }
__device__ __forceinline__ void st(float* p, long i, float x) { p[i] = x; }
__device__ __forceinline__ void st(bf16s* p, long i, float x) { p[i].v = f2bf(x); }

// ---- gauge fixing and features -------------------------------------------------
// links: [B][2][H*W] complex128 (canonical U(1) layout per configuration);
// theta_mu(x) = arg U_mu(x).
__device__ __forceinline__ double link_angle(const double2* U, int b, int mu, long HW, long p) {
  const double2 u = U[((long)b * 2 + mu) * HW + p];
  return atan2(u.y, u.x);
}

// phi at every site of a block: 0 at the block origin, along the first
// column phi(y) = phi(y - 1) + theta_2(y - 1), along rows phi(x) = phi(x - 1) + theta_1(x - 1)
__global__ void tree_phase_kernel(const double2* __restrict__ U, double* __restrict__ phi, int H, int W, int B) {
  const int nbx = W / BLK, nby = H / BLK;
  const long nblk = (long)B * nbx * nby;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nblk; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / (nbx * nby));
    const int j = (int)(t - (long)b * nbx * nby);
    const int y0 = (j / nbx) * BLK, x0 = (j % nbx) * BLK;
    const long HW = (long)H * W;
    double* ph = phi + (long)b * HW;
    for (int yy = 0; yy < BLK; ++yy)
      for (int xx = 0; xx < BLK; ++xx) {
        const int y = y0 + yy, x = x0 + xx;
        double v;
        if (xx == 0) v = (yy == 0) ? 0.0 : ph[(long)(y - 1) * W + x] + link_angle(U, b, 1, HW, (long)(y - 1) * W + x);
        else v = ph[(long)y * W + x - 1] + link_angle(U, b, 0, HW, (long)y * W + x - 1);
        ph[(long)y * W + x] = v;
      }
  }
}

template <typename TS>
__global__ void features_kernel(const double2* __restrict__ U, const double* __restrict__ phi, TS* __restrict__ feat,
                                int H, int W, int B) {
  const long HW = (long)H * W;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < B * HW; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / HW);
    const long p = t - (long)b * HW;
    const int y = (int)(p / W), x = (int)(p - (long)y * W);
    const double* ph = phi + (long)b * HW;
    const double f0 = ph[p];
    const double a1 = f0 + link_angle(U, b, 0, HW, p) - ph[(long)y * W + (x + 1) % W];
    const double a2 = f0 + link_angle(U, b, 1, HW, p) - ph[(long)((y + 1) % H) * W + x];
    TS* o = feat + (long)b * 4 * HW;
    st(o, p, (float)cos(a1));
    st(o, HW + p, (float)sin(a1));
    st(o, 2 * HW + p, (float)cos(a2));
    st(o, 3 * HW + p, (float)sin(a2));
  }
}

// targets in the fixed gauge: t'(x) = exp(i phi(x)) t(x); vecs canonical [B][NVEC][V][2]
__global__ void targets_kernel(const double2* __restrict__ vecs, const double* __restrict__ phi,
                               double2* __restrict__ tgt, long HW, int B) {
  const long tot = (long)B * NVEC * HW;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long)gridDim.x * blockDim.x) {
    const int b = (int)(t / (NVEC * HW));
    const long p = t % HW;
    const double f = phi[(long)b * HW + p];
    const double c = cos(f), s = sin(f);
    for (int sp = 0; sp < 2; ++sp) {
      const double2 v = vecs[t * 2 + sp];
      tgt[t * 2 + sp] = make_double2(c * v.x - s * v.y, c * v.y + s * v.x);
    }
  }
}

// proposals back in the original gauge: v(x) = exp(-i phi(x)) (y_re + i y_im), canonical [NVEC][V][2]
template <typename TS>
__global__ void proposals_kernel(const TS* __restrict__ y, const double* __restrict__ phi, double2* __restrict__ out,
                                 long HW) {
  const long tot = (long)NVEC * HW;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (long)gridDim.x * blockDim.x) {
    const int k = (int)(t / HW);
    const long p = t - (long)k * HW;
    const double c = cos(phi[p]), s = sin(phi[p]);
    for (int sp = 0; sp < 2; ++sp) {
      const double re = ld(y, (long)(4 * k + 2 * sp) * HW + p), im = ld(y, (long)(4 * k + 2 * sp + 1) * HW + p);
      out[t * 2 + sp] = make_double2(c * re + s * im, c * im - s * re);
    }
  }
}

// ---- 3x3 periodic convolution ---------------------------------------------------
// y[b][o][p] = bias[o] + sum_{c,k} W[o][c][k] x[b][c][p + d_k] (d_k = (k/3 - 1, k%3 - 1)),
// tile of 16 x 16 pixels x 16 output channels per 256-thread block, input
// channels staged through LDS 8 at a time (with a one-site halo).
// FLIP: the data gradient, dx[c] = sum_o W[o][c][8 - k] dy[o][p + d_k]
// (weights read transposed and flipped; "Cin" = forward Cout).
// ACT: forward applies tanh; backward multiplies by 1 - a^2 of `act`.
constexpr int TILE = 16, OC = 16, CC = 8;

template <typename TI, typename TO, typename TW, bool FLIP, bool ACT>
__global__ __launch_bounds__(256) void conv3x3_kernel(const TI* __restrict__ x, const TW* __restrict__ Wt,
                                                      const float* __restrict__ bias, TO* __restrict__ y,
                                                      const void* __restrict__ actv, int Cin, int Cout, int H, int W,
                                                      int actbf16) {
  __shared__ float xs[CC][TILE + 2][TILE + 2];
  __shared__ float ws[OC][CC][9];
  const int b = blockIdx.z;
  const int ntx = W / TILE;
  const int tx0 = (blockIdx.x % ntx) * TILE, ty0 = (blockIdx.x / ntx) * TILE;
  const int o0 = blockIdx.y * OC;
  const int t = threadIdx.x;
  const int py = t / TILE, px = t % TILE;
  const long HW = (long)H * W;
  float acc[OC];
#pragma unroll
  for (int o = 0; o < OC; ++o) acc[o] = (bias && o0 + o < Cout) ? bias[o0 + o] : 0.f;
  for (int c0 = 0; c0 < Cin; c0 += CC) {
    const int cc = min(CC, Cin - c0);
    for (int idx = t; idx < CC * (TILE + 2) * (TILE + 2); idx += 256) {
      const int c = idx / ((TILE + 2) * (TILE + 2));
      const int r = idx - c * (TILE + 2) * (TILE + 2);
      const int yy = r / (TILE + 2), xx = r - yy * (TILE + 2);
      float v = 0.f;
      if (c < cc) {
        const int gy = (ty0 + yy - 1 + H) % H, gx = (tx0 + xx - 1 + W) % W;
        v = ld(x, ((long)b * Cin + c0 + c) * HW + (long)gy * W + gx);
      }
      xs[c][yy][xx] = v;
    }
    for (int idx = t; idx < OC * CC * 9; idx += 256) {
      const int o = idx / (CC * 9);
      const int r = idx - o * CC * 9;
      const int c = r / 9, k = r - c * 9;
      float v = 0.f;
      if (c < cc && o0 + o < Cout) {
        // forward: W[o][c][k] with shape [Cout][Cin][9]; FLIP: W[c][o][8-k] with shape [Cin][Cout][9]
        v = FLIP ? ld(Wt, ((long)(c0 + c) * Cout + o0 + o) * 9 + (8 - k)) : ld(Wt, ((long)(o0 + o) * Cin + c0 + c) * 9 + k);
      }
      ws[o][c][k] = v;
    }
    __syncthreads();
    for (int c = 0; c < cc; ++c) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float v = xs[c][py + k / 3][px + k % 3];
#pragma unroll
        for (int o = 0; o < OC; ++o) acc[o] = fmaf(ws[o][c][k], v, acc[o]);
      }
    }
    __syncthreads();
  }
  const long p = (long)(ty0 + py) * W + tx0 + px;
#pragma unroll
  for (int o = 0; o < OC; ++o) {
    if (o0 + o >= Cout) continue;
    float v = acc[o];
    const long i = ((long)b * Cout + o0 + o) * HW + p;
    if (ACT) {
      if (FLIP) {
        const float a = actbf16 ? ld((const bf16s*)actv, i) : ld((const float*)actv, i);
        v *= (1.f - a * a);
      } else {
        v = tanhf(v);
      }
    }
    st(y, i, v);
  }
}

// dW[o][c][k] += sum_{b,p} dy[b][o][p] x[b][c][p + d_k];  db[o] += sum dy[b][o][p]
// block: 16 output channels x 8 input channels, a run of pixel tiles; partial
// sums added to the FP32 gradient with atomics.
constexpr int WG_TILES = 8;
template <typename TS>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const TS* __restrict__ x, const float* __restrict__ dy,
                                                            float* __restrict__ dW, float* __restrict__ db, int Cin,
                                                            int Cout, int H, int W, int B) {
  __shared__ float xs[CC][TILE + 2][TILE + 2];
  __shared__ float ds[OC][TILE * TILE];
  const int o0 = blockIdx.y * OC, c0 = blockIdx.z * CC;
  const int cc = min(CC, Cin - c0);
  const int t = threadIdx.x;
  const long HW = (long)H * W;
  const int ntx = W / TILE, nty = H / TILE;
  const long ntiles = (long)B * ntx * nty;
  // thread t owns output channel o = t / 16 and pairs q = t % 16 + 16 j of (c, k)
  const int o = t / 16, q0 = t % 16;
  float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  for (long tile = (long)blockIdx.x * WG_TILES; tile < min(ntiles, (long)(blockIdx.x + 1) * WG_TILES); ++tile) {
    const int b = (int)(tile / (ntx * nty));
    const int tt = (int)(tile - (long)b * ntx * nty);
    const int tx0 = (tt % ntx) * TILE, ty0 = (tt / ntx) * TILE;
    for (int idx = t; idx < CC * (TILE + 2) * (TILE + 2); idx += 256) {
      const int c = idx / ((TILE + 2) * (TILE + 2));
      const int r = idx - c * (TILE + 2) * (TILE + 2);
      const int yy = r / (TILE + 2), xx = r - yy * (TILE + 2);
      float v = 0.f;
      if (c < cc) {
        const int gy = (ty0 + yy - 1 + H) % H, gx = (tx0 + xx - 1 + W) % W;
        v = ld(x, ((long)b * Cin + c0 + c) * HW + (long)gy * W + gx);
      }
      xs[c][yy][xx] = v;
    }
    for (int idx = t; idx < OC * TILE * TILE; idx += 256) {
      const int oo = idx / (TILE * TILE), pp = idx - oo * TILE * TILE;
      ds[oo][pp] = (o0 + oo < Cout) ? dy[((long)b * Cout + o0 + oo) * HW + (long)(ty0 + pp / TILE) * W + tx0 + pp % TILE]
                                    : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int q = q0 + 16 * j;
      if (q < cc * 9) {
        const int c = q / 9, k = q - c * 9;
        float s = 0.f;
        for (int pp = 0; pp < TILE * TILE; ++pp) s = fmaf(ds[o][pp], xs[c][pp / TILE + k / 3][pp % TILE + k % 3], s);
        acc[j] += s;
      }
    }
    if (blockIdx.z == 0 && q0 == 0)
      for (int pp = 0; pp < TILE * TILE; ++pp) bacc += ds[o][pp];
    __syncthreads();
  }
  if (o0 + o < Cout) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const int q = q0 + 16 * j;
      if (q < cc * 9) atomicAdd(&dW[((long)(o0 + o) * Cin + c0 + q / 9) * 9 + q % 9], acc[j]);
    }
    if (blockIdx.z == 0 && q0 == 0) atomicAdd(&db[o0 + o], bacc);
  }
}

// ---- the same convolutions on the matrix cores (bfloat16 storage mode) -----------
// Implicit GEMM on v_mfma_f32_16x16x16_bf16 (bf16 operands, FP32 accumulation):
// Y[o][p] = sum_kk A[o][kk] B[kk][p] with kk = tap * Cin + c, tap-major, so
// the four K values a lane supplies are four consecutive channels of one tap.
// Operand layout of the 16x16x16 instruction: lane l gives A[l % 16][4 (l/16) .. +3]
// and B[4 (l/16) .. +3][l % 16] and receives D[4 (l/16) + r][l % 16], r < 4.
typedef short mf_v4s __attribute__((ext_vector_type(4)));
typedef float mf_v4f __attribute__((ext_vector_type(4)));
constexpr int MT = 16;     // pixel tile MT x MT
constexpr int MOC = 32;    // output channels per block (two waves of 16)
constexpr int MCMAX = 64;  // largest channel count

__device__ __forceinline__ uint16_t to_bf(float v) { return f2bf(v); }
__device__ __forceinline__ float ldf(const float* p, long i) { return p[i]; }
__device__ __forceinline__ float ldf(const bf16s* p, long i) { return bf2f(p[i].v); }

// Forward (FLIP = false): y[o] = act(bias[o] + sum_{c,tap} W[o][c][tap] x[c][p + d_tap]).
// Data gradient (FLIP): y[c] = (1 - a^2) sum_{o,tap} W[o][c][8 - tap] dy[o][p + d_tap]
// ("Cin" = forward Cout).  Block: a 16 x 16 pixel tile and 32 output
// channels; wave w takes channels 16 (w & 1) .. +15 and pixel rows
// 8 (w >> 1) .. +7 (eight 16-pixel MFMA columns, one per row).  The input tile
// with its one-site halo and the block's weights sit in LDS channel-fastest,
// so each operand is one 8-byte read.  Cin a multiple of 4 (<= 64), Cout of
// 16, H and W of 16.
template <typename TI, typename TO, bool FLIP, bool ACT>
__global__ __launch_bounds__(256) void conv3x3_mfma_kernel(const TI* __restrict__ x, const bf16s* __restrict__ Wt,
                                                           const float* __restrict__ bias, TO* __restrict__ y,
                                                           const bf16s* __restrict__ actv, int Cin, int Cout, int H,
                                                           int W) {
  // input channels staged 16 at a time (24.5 KB of LDS, six blocks per CU);
  // channel stride MCK + 4: the 16 rows of an operand read fall in distinct
  // LDS banks and every 4-channel group stays 8-byte aligned
  constexpr int MCK = 16, CS = MCK + 4, SU = 8;
  __shared__ __align__(16) uint16_t xs[(MT + 2) * (MT + 2) * CS];
  __shared__ __align__(16) uint16_t ws[MOC * 9 * CS];
  const int b = blockIdx.z;
  const int ntx = W / MT;
  const int tx0 = (blockIdx.x % ntx) * MT, ty0 = (blockIdx.x / ntx) * MT;
  const int o0 = blockIdx.y * MOC;
  const int t = threadIdx.x;
  const long HW = (long)H * W;
  const int wv = t >> 6, lane = t & 63;
  const int og = wv & 1, ph = wv >> 1;
  const int lr = lane & 15, lg = lane >> 4;
  constexpr int NT = MT * MT / 2 / 16;  // MFMA columns per wave
  mf_v4f acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = mf_v4f{0.f, 0.f, 0.f, 0.f};
  for (int cb = 0; cb < Cin; cb += MCK) {
    const int cc = min(MCK, Cin - cb);
    __syncthreads();
    // stage (SU loads in flight per thread before their LDS stores)
    const int nx = cc * (MT + 2) * (MT + 2);
    for (int i0 = t; i0 < nx; i0 += 256 * SU) {
      float v[SU];
      int dst[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = i0 + u * 256;
        dst[u] = -1;
        v[u] = 0.f;
        if (idx < nx) {
          const int c = idx / ((MT + 2) * (MT + 2)), pos = idx - c * (MT + 2) * (MT + 2);
          const int yy = pos / (MT + 2), xx = pos - yy * (MT + 2);
          int gy = ty0 + yy - 1, gx = tx0 + xx - 1;
          gy = gy < 0 ? gy + H : (gy >= H ? gy - H : gy);
          gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
          v[u] = ldf(x, ((long)b * Cin + cb + c) * HW + (long)gy * W + gx);
          dst[u] = pos * CS + c;
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (dst[u] >= 0) xs[dst[u]] = to_bf(v[u]);
    }
    const int nw = MOC * cc * 9;
    for (int i0 = t; i0 < nw; i0 += 256 * SU) {
      uint16_t v[SU];
      int dst[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = i0 + u * 256;
        dst[u] = -1;
        v[u] = 0;
        if (idx < nw) {
          const int ol = idx / (cc * 9), r = idx - ol * cc * 9;
          const int c = r / 9, k = r - c * 9;
          if (o0 + ol < Cout)
            v[u] = FLIP ? Wt[((long)(cb + c) * Cout + o0 + ol) * 9 + (8 - k)].v
                        : Wt[((long)(o0 + ol) * Cin + cb + c) * 9 + k].v;
          dst[u] = (ol * 9 + k) * CS + c;
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (dst[u] >= 0) ws[dst[u]] = v[u];
    }
    __syncthreads();
    const int c = 4 * lg;
    const bool on = c < cc;  // lanes past the chunk (Cin = 4) supply zeros; the MFMA runs in every lane
    const mf_v4s z = mf_v4s{0, 0, 0, 0};
    for (int tap = 0; tap < 9; ++tap) {
      const int ty = tap / 3, tx = tap - ty * 3;
      const mf_v4s a = on ? *reinterpret_cast<const mf_v4s*>(&ws[((og * 16 + lr) * 9 + tap) * CS + c]) : z;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int pp = ph * (NT * 16) + nt * 16 + lr;
        const int py = pp / MT, px = pp - py * MT;
        const mf_v4s bv = on ? *reinterpret_cast<const mf_v4s*>(&xs[((py + ty) * (MT + 2) + px + tx) * CS + c]) : z;
        acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[nt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int pp = ph * (NT * 16) + nt * 16 + lr;
    const int py = pp / MT, px = pp - py * MT;
    const long pix = (long)(ty0 + py) * W + tx0 + px;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = o0 + og * 16 + 4 * lg + r;
      if (o >= Cout) continue;
      float v = acc[nt][r];
      const long i = ((long)b * Cout + o) * HW + pix;
      if (!FLIP && bias) v += bias[o];
      if (ACT) {
        if (FLIP) {
          const float av = bf2f(actv[i].v);
          v *= 1.f - av * av;
        } else {
          v = tanhf(v);
        }
      }
      st(y, i, v);
    }
  }
}

// dW[o][c][tap] += sum_{b,p} dy[b][o][p] x[b][c][p + d_tap], db[o] += sum dy[b][o][p]:
// M = o, N = c, K = pixels.  One wave per (16 output, 16 input channels) for
// all nine taps, over a run of 16 x 16 pixel tiles; dy (FP32, rounded to bf16)
// and x staged in LDS pixel-fastest; partial sums added to the FP32 gradient
// with atomics.
constexpr int MWG_TILES = 4;
template <typename TS>
__global__ __launch_bounds__(64) void conv3x3_wgrad_mfma_kernel(const TS* __restrict__ x, const float* __restrict__ dy,
                                                                float* __restrict__ dW, float* __restrict__ db,
                                                                int Cin, int Cout, int H, int W, int B) {
  __shared__ __align__(16) uint16_t ds[16][MT * MT + 4];  // padded rows: the 16 lanes of a read hit distinct banks
  __shared__ uint16_t xs2[16][(MT + 2) * (MT + 2) + 2];
  const int ncg = (Cin + 15) / 16;
  const int o0 = (blockIdx.y / ncg) * 16, c0 = (blockIdx.y % ncg) * 16;
  const int lane = threadIdx.x, lr = lane & 15, lg = lane >> 4;
  const long HW = (long)H * W;
  const int ntx = W / MT, nty = H / MT;
  const long ntiles = (long)B * ntx * nty;
  mf_v4f acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = mf_v4f{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  const long t_end = min(ntiles, (long)(blockIdx.x + 1) * MWG_TILES);
  for (long tile = (long)blockIdx.x * MWG_TILES; tile < t_end; ++tile) {
    const int b = (int)(tile / (ntx * nty));
    const int tt = (int)(tile - (long)b * ntx * nty);
    const int tx0 = (tt % ntx) * MT, ty0 = (tt / ntx) * MT;
    __syncthreads();
    // staging with SU loads in flight per lane
    constexpr int SU = 8;
    for (int j0 = 0; j0 < 16 * MT * MT / 64; j0 += SU) {
      float v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = lane + 64 * (j0 + u);
        const int ol = idx / (MT * MT), pp = idx - ol * MT * MT;
        v[u] = (o0 + ol < Cout) ? dy[((long)b * Cout + o0 + ol) * HW + (long)(ty0 + pp / MT) * W + tx0 + pp % MT] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = lane + 64 * (j0 + u);
        const int ol = idx / (MT * MT), pp = idx - ol * MT * MT;
        ds[ol][pp] = to_bf(v[u]);
      }
    }
    const int nx2 = 16 * (MT + 2) * (MT + 2);
    for (int i0 = lane; i0 < nx2; i0 += 64 * SU) {
      float v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = i0 + 64 * u;
        v[u] = 0.f;
        if (idx < nx2) {
          const int cl = idx / ((MT + 2) * (MT + 2)), pos = idx - cl * (MT + 2) * (MT + 2);
          const int yy = pos / (MT + 2), xx = pos - yy * (MT + 2);
          if (c0 + cl < Cin) {
            int gy = ty0 + yy - 1, gx = tx0 + xx - 1;
            gy = gy < 0 ? gy + H : (gy >= H ? gy - H : gy);
            gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
            v[u] = ldf(x, ((long)b * Cin + c0 + cl) * HW + (long)gy * W + gx);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int idx = i0 + 64 * u;
        if (idx < nx2) {
          const int cl = idx / ((MT + 2) * (MT + 2)), pos = idx - cl * (MT + 2) * (MT + 2);
          xs2[cl][pos] = to_bf(v[u]);
        }
      }
    }
    __syncthreads();
    if (c0 == 0) {
      // bias gradient from the staged tile: lane (o = lane / 4, quarter lane % 4)
      // sums 64 pixels, then the four quarters are added
      const int ob = lane >> 2, q = lane & 3;
      float sb = 0.f;
      for (int pp = q * (MT * MT / 4); pp < (q + 1) * (MT * MT / 4); ++pp) sb += bf2f(ds[ob][pp]);
      sb += __shfl_xor(sb, 1);
      sb += __shfl_xor(sb, 2);
      if (q == 0) bacc += sb;  // lane 4 ob holds output channel ob's sum
    }
#pragma unroll
    for (int ks = 0; ks < MT * MT / 16; ++ks) {
      const int p0 = ks * 16 + 4 * lg;  // this lane's 4 pixels (one tile row: MT is a multiple of 4)
      const mf_v4s a = *reinterpret_cast<const mf_v4s*>(&ds[lr][p0]);
      const int py = p0 / MT, px = p0 - py * MT;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int ty = tap / 3, tx = tap - ty * 3;
        const uint16_t* xr = &xs2[lr][(py + ty) * (MT + 2) + px + tx];
        const mf_v4s bv = mf_v4s{(short)xr[0], (short)xr[1], (short)xr[2], (short)xr[3]};
        acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[tap], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = o0 + 4 * lg + r, c = c0 + lr;
      if (o < Cout && c < Cin) atomicAdd(&dW[((long)o * Cin + c) * 9 + tap], acc[tap][r]);
    }
  if (c0 == 0 && (lane & 3) == 0 && o0 + (lane >> 2) < Cout) atomicAdd(&db[o0 + (lane >> 2)], bacc);
}

// ---- projection loss -------------------------------------------------------------
// one 64-lane workgroup per (block j, chirality s, configuration b); FP64.
// V[i][a]: prediction a at block site i, T[i][k]: normalised target k,
// G = V^dag V + eps (Cholesky in LDS), U = V^dag T, W = G^-1 U (column k is
// w_k), M = W W^dag, loss_js = sum_k (1 - u_k^dag w_k) and
// dL/d(conj V) = -T W^dag + V M (Wirtinger; real gradients 2 Re, 2 Im).
template <typename TS>
__global__ __launch_bounds__(64) void loss_kernel(const TS* __restrict__ yout, const double2* __restrict__ tgt,
                                                  float* __restrict__ dout, double* __restrict__ loss, int H, int W,
                                                  double scale) {
  __shared__ double2 Vs[16][NVEC], Ts[16][NVEC], G[NVEC][NVEC], Um[NVEC][NVEC], Wm[NVEC][NVEC], Mm[NVEC][NVEC];
  __shared__ double tn[NVEC], lpart[NVEC];
  const int nbx = W / BLK;
  const int s = blockIdx.x & 1, j = blockIdx.x >> 1, b = blockIdx.y;
  const int y0 = (j / nbx) * BLK, x0 = (j % nbx) * BLK;
  const long HW = (long)H * W;
  const int t = threadIdx.x;
  for (int e = t; e < 16 * NVEC; e += 64) {
    const int i = e / NVEC, k = e % NVEC;
    const long pix = (long)(y0 + i / BLK) * W + x0 + i % BLK;
    const long base = ((long)b * 4 * NVEC + 4 * k + 2 * s) * HW + pix;
    Vs[i][k] = make_double2(ld(yout, base), ld(yout, base + HW));
    Ts[i][k] = tgt[(((long)b * NVEC + k) * HW + pix) * 2 + s];
  }
  __syncthreads();
  if (t < NVEC) {
    double nn = 0.0;
    for (int i = 0; i < 16; ++i) nn += Ts[i][t].x * Ts[i][t].x + Ts[i][t].y * Ts[i][t].y;
    tn[t] = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < 16 * NVEC; e += 64) {
    const int i = e / NVEC, k = e % NVEC;
    Ts[i][k] = make_double2(Ts[i][k].x * tn[k], Ts[i][k].y * tn[k]);
  }
  __syncthreads();
  {
    const int a = t / NVEC, c = t % NVEC;  // G[a][c] and U[a][c]
    double gr = (a == c) ? LOSS_EPS : 0.0, gi = 0.0, ur = 0.0, ui = 0.0;
    for (int i = 0; i < 16; ++i) {
      const double2 p = Vs[i][a], q = Vs[i][c], r = Ts[i][c];
      gr += p.x * q.x + p.y * q.y;
      gi += p.x * q.y - p.y * q.x;
      ur += p.x * r.x + p.y * r.y;
      ui += p.x * r.y - p.y * r.x;
    }
    G[a][c] = make_double2(gr, gi);
    Um[a][c] = make_double2(ur, ui);
  }
  __syncthreads();
  if (t == 0) {  // G = L L^dag, L lower, stored in place
    for (int c = 0; c < NVEC; ++c) {
      double d = G[c][c].x;
      for (int q = 0; q < c; ++q) d -= G[c][q].x * G[c][q].x + G[c][q].y * G[c][q].y;
      d = sqrt(d > 1e-300 ? d : 1e-300);
      G[c][c] = make_double2(d, 0.0);
      for (int r = c + 1; r < NVEC; ++r) {
        double re = G[r][c].x, im = G[r][c].y;
        for (int q = 0; q < c; ++q) {  // -= L[r][q] conj(L[c][q])
          re -= G[r][q].x * G[c][q].x + G[r][q].y * G[c][q].y;
          im -= G[r][q].y * G[c][q].x - G[r][q].x * G[c][q].y;
        }
        G[r][c] = make_double2(re / d, im / d);
      }
    }
  }
  __syncthreads();
  if (t < NVEC) {  // column k = t: L z = u_k, L^dag w_k = z
    const int k = t;
    double2 z[NVEC];
    for (int r = 0; r < NVEC; ++r) {
      double re = Um[r][k].x, im = Um[r][k].y;
      for (int q = 0; q < r; ++q) {
        re -= G[r][q].x * z[q].x - G[r][q].y * z[q].y;
        im -= G[r][q].x * z[q].y + G[r][q].y * z[q].x;
      }
      z[r] = make_double2(re / G[r][r].x, im / G[r][r].x);
    }
    for (int r = NVEC - 1; r >= 0; --r) {
      double re = z[r].x, im = z[r].y;
      for (int q = r + 1; q < NVEC; ++q) {  // -= conj(L[q][r]) w[q]
        re -= G[q][r].x * z[q].x + G[q][r].y * z[q].y;
        im -= G[q][r].x * z[q].y - G[q][r].y * z[q].x;
      }
      z[r] = make_double2(re / G[r][r].x, im / G[r][r].x);
    }
    double uw = 0.0;
    for (int a = 0; a < NVEC; ++a) {
      Wm[a][k] = z[a];
      uw += Um[a][k].x * z[a].x + Um[a][k].y * z[a].y;
    }
    lpart[k] = 1.0 - uw;
  }
  __syncthreads();
  if (t == 0) {
    double l = 0.0;
    for (int k = 0; k < NVEC; ++k) l += lpart[k];
    atomicAdd(loss, l * scale);
  }
  if (dout == nullptr) return;
  {
    const int a = t / NVEC, c = t % NVEC;  // M[a][c] = sum_k w_k[a] conj(w_k[c])
    double re = 0.0, im = 0.0;
    for (int k = 0; k < NVEC; ++k) {
      const double2 p = Wm[a][k], q = Wm[c][k];
      re += p.x * q.x + p.y * q.y;
      im += p.y * q.x - p.x * q.y;
    }
    Mm[a][c] = make_double2(re, im);
  }
  __syncthreads();
  for (int e = t; e < 16 * NVEC; e += 64) {
    const int i = e / NVEC, a = e % NVEC;
    double re = 0.0, im = 0.0;
    for (int k = 0; k < NVEC; ++k) {  // - t_k[i] conj(w_k[a])
      const double2 p = Ts[i][k], q = Wm[a][k];
      re -= p.x * q.x + p.y * q.y;
      im -= p.y * q.x - p.x * q.y;
    }
    for (int c = 0; c < NVEC; ++c) {  // + V[i][c] M[c][a]
      const double2 p = Vs[i][c], q = Mm[c][a];
      re += p.x * q.x - p.y * q.y;
      im += p.x * q.y + p.y * q.x;
    }
    const long pix = (long)(y0 + i / BLK) * W + x0 + i % BLK;
    const long base = ((long)b * 4 * NVEC + 4 * a + 2 * s) * HW + pix;
    dout[base] = (float)(2.0 * re * scale);
    dout[base + HW] = (float)(2.0 * im * scale);
  }
}

__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, long n, float lr, float b1, float b2, float eps, float c1, float c2,
                            void* __restrict__ ws, int bf16) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (ws == nullptr) continue;
    if (bf16) st((bf16s*)ws, i, wi);
    else st((float*)ws, i, wi);
  }
}

__global__ void widen_kernel(const bf16s* __restrict__ in, float* __restrict__ out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) out[i] = ld(in, i);
}

__global__ void cast_kernel(const float* __restrict__ in, void* __restrict__ out, long n, int bf16) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    if (bf16) st((bf16s*)out, i, in[i]);
    else st((float*)out, i, in[i]);
  }
}

inline unsigned nb(long n) {
  long b = (n + 255) / 256;
  if (b > (1L << 20)) b = 1L << 20;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

struct amg_cnn {
  int bf16 = 1;
  long nW[NL], nB[NL];
  Buf W32[NL], B32[NL], Ws[NL], mW[NL], vW[NL], mB[NL], vB[NL], gW[NL], gB[NL];
  Buf act[NL + 1], grad[NL + 1], phi, tgt, loss;
  double* loss_host = nullptr;
  long cap = 0;  // B * H * W capacity of the work buffers
  long step = 0;
  size_t ssz() const { return bf16 ? 2 : 4; }
  ~amg_cnn() {
    if (loss_host) (void)hipHostFree(loss_host);
  }
};

namespace {

using Cnn = amg_cnn;

long total_params() {
  long n = 0;
  for (int l = 0; l < NL; ++l) n += (long)CH[l + 1] * CH[l] * 9 + CH[l + 1];
  return n;
}

void cnn_ensure(Cnn& N, int B, int H, int W) {
  const long need = (long)B * H * W;
  if (need <= N.cap) return;
  for (int l = 0; l <= NL; ++l) {
    N.act[l].ensure(need * CH[l] * N.ssz());
    N.grad[l].ensure(need * CH[l] * sizeof(float));
  }
  N.phi.ensure(need * sizeof(double));
  N.tgt.ensure(need * NVEC * 2 * sizeof(double2));
  N.cap = need;
}

template <typename TS>
void forward(Cnn& N, const double2* U, int B, int H, int W, hipStream_t st) {
  const long nblk = (long)B * (W / BLK) * (H / BLK);
  hipLaunchKernelGGL(tree_phase_kernel, dim3(nb(nblk)), dim3(256), 0, st, U, N.phi.as<double>(), H, W, B);
  hipLaunchKernelGGL((features_kernel<TS>), dim3(nb((long)B * H * W)), dim3(256), 0, st, U, N.phi.as<double>(),
                     N.act[0].as<TS>(), H, W, B);
  for (int l = 0; l < NL; ++l) {
    if constexpr (std::is_same<TS, bf16s>::value) {  // bf16 storage: implicit GEMM on the matrix cores
      dim3 gm((W / MT) * (H / MT), (CH[l + 1] + MOC - 1) / MOC, B);
      if (l < NL - 1)
        hipLaunchKernelGGL((conv3x3_mfma_kernel<bf16s, bf16s, false, true>), gm, dim3(256), 0, st,
                           N.act[l].as<bf16s>(), N.Ws[l].as<bf16s>(), N.B32[l].as<float>(), N.act[l + 1].as<bf16s>(),
                           nullptr, CH[l], CH[l + 1], H, W);
      else
        hipLaunchKernelGGL((conv3x3_mfma_kernel<bf16s, bf16s, false, false>), gm, dim3(256), 0, st,
                           N.act[l].as<bf16s>(), N.Ws[l].as<bf16s>(), N.B32[l].as<float>(), N.act[l + 1].as<bf16s>(),
                           nullptr, CH[l], CH[l + 1], H, W);
      continue;
    }
    dim3 grid((W / TILE) * (H / TILE), (CH[l + 1] + OC - 1) / OC, B);
    if (l < NL - 1)
      hipLaunchKernelGGL((conv3x3_kernel<TS, TS, TS, false, true>), grid, dim3(256), 0, st, N.act[l].as<TS>(),
                         N.Ws[l].as<TS>(), N.B32[l].as<float>(), N.act[l + 1].as<TS>(), nullptr, CH[l], CH[l + 1],
                         H, W, 0);
    else
      hipLaunchKernelGGL((conv3x3_kernel<TS, TS, TS, false, false>), grid, dim3(256), 0, st, N.act[l].as<TS>(),
                         N.Ws[l].as<TS>(), N.B32[l].as<float>(), N.act[l + 1].as<TS>(), nullptr, CH[l], CH[l + 1],
                         H, W, 0);
  }
}

// mean loss over (configurations, blocks, chiralities, target vectors) and,
// when grads, its gradient with respect to every parameter into gW, gB
template <typename TS>
double loss_and_grads(Cnn& N, const double2* U, const double2* vecs, int B, int H, int W, bool grads,
                      hipStream_t st) {
  forward<TS>(N, U, B, H, W, st);
  const long HW = (long)H * W;
  hipLaunchKernelGGL(targets_kernel, dim3(nb((long)B * NVEC * HW)), dim3(256), 0, st, vecs, N.phi.as<double>(),
                     N.tgt.as<double2>(), HW, B);
  HIPC(hipMemsetAsync(N.loss.p, 0, sizeof(double), st));
  const long nbj = HW / (BLK * BLK);
  const double scale = 1.0 / ((double)B * nbj * 2 * NVEC);
  hipLaunchKernelGGL((loss_kernel<TS>), dim3((unsigned)(2 * nbj), (unsigned)B), dim3(64), 0, st, N.act[NL].as<TS>(),
                     N.tgt.as<double2>(), grads ? N.grad[NL].as<float>() : nullptr, N.loss.as<double>(), H, W, scale);
  if (grads) {
    for (int l = NL - 1; l >= 0; --l) {
      HIPC(hipMemsetAsync(N.gW[l].p, 0, sizeof(float) * N.nW[l], st));
      HIPC(hipMemsetAsync(N.gB[l].p, 0, sizeof(float) * N.nB[l], st));
      if constexpr (std::is_same<TS, bf16s>::value) {
        const long mt = (long)B * (H / MT) * (W / MT);
        dim3 gmw((unsigned)((mt + MWG_TILES - 1) / MWG_TILES), (unsigned)(((CH[l + 1] + 15) / 16) * ((CH[l] + 15) / 16)));
        hipLaunchKernelGGL((conv3x3_wgrad_mfma_kernel<bf16s>), gmw, dim3(64), 0, st, N.act[l].as<bf16s>(),
                           N.grad[l + 1].as<float>(), N.gW[l].as<float>(), N.gB[l].as<float>(), CH[l], CH[l + 1], H, W,
                           B);
        if (l > 0) {
          dim3 gm((W / MT) * (H / MT), (CH[l] + MOC - 1) / MOC, B);
          hipLaunchKernelGGL((conv3x3_mfma_kernel<float, float, true, true>), gm, dim3(256), 0, st,
                             N.grad[l + 1].as<float>(), N.Ws[l].as<bf16s>(), (const float*)nullptr,
                             N.grad[l].as<float>(), N.act[l].as<bf16s>(), CH[l + 1], CH[l], H, W);
        }
        continue;
      }
      const long ntiles = (long)B * (H / TILE) * (W / TILE);
      dim3 gw((unsigned)((ntiles + WG_TILES - 1) / WG_TILES), (CH[l + 1] + OC - 1) / OC, (CH[l] + CC - 1) / CC);
      hipLaunchKernelGGL((conv3x3_wgrad_kernel<TS>), gw, dim3(256), 0, st, N.act[l].as<TS>(), N.grad[l + 1].as<float>(),
                         N.gW[l].as<float>(), N.gB[l].as<float>(), CH[l], CH[l + 1], H, W, B);
      if (l > 0) {
        dim3 grid((W / TILE) * (H / TILE), (CH[l] + OC - 1) / OC, B);
        hipLaunchKernelGGL((conv3x3_kernel<float, float, TS, true, true>), grid, dim3(256), 0, st,
                           N.grad[l + 1].as<float>(), N.Ws[l].as<TS>(), (const float*)nullptr, N.grad[l].as<float>(),
                           (const void*)N.act[l].p, CH[l + 1], CH[l], H, W, N.bf16);
      }
    }
  }
  HIPC(hipGetLastError());
  HIPC(hipMemcpyAsync(N.loss_host, N.loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return *N.loss_host;
}

void upload_params(Cnn& N, const float* host) {
  long off = 0;
  for (int l = 0; l < NL; ++l) {
    HIPC(hipMemcpy(N.W32[l].p, host + off, sizeof(float) * N.nW[l], hipMemcpyHostToDevice));
    off += N.nW[l];
    HIPC(hipMemcpy(N.B32[l].p, host + off, sizeof(float) * N.nB[l], hipMemcpyHostToDevice));
    off += N.nB[l];
    hipLaunchKernelGGL(cast_kernel, dim3(nb(N.nW[l])), dim3(256), 0, nullptr, N.W32[l].as<float>(), N.Ws[l].p, N.nW[l],
                       N.bf16);
  }
  HIPC(hipGetLastError());
  HIPC(hipDeviceSynchronize());
}

void check_lattice(int B, int L1, int L2) {
  if (B < 1 || L1 < TILE || L2 < TILE || L1 % TILE || L2 % TILE)
    fail(AMG_ERR_SHAPE, "the network needs B >= 1 and lattice extents that are multiples of 16");
  if ((long)B * L1 * L2 > (1L << 28)) fail(AMG_ERR_SHAPE, "batch too large");
}

void check_params_finite(const float* p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) fail(AMG_ERR_NAN, "non-finite network parameter");
}

}  // namespace

extern "C" {

long long amg_cnn_num_params(void) { return total_params(); }

amg_status amg_cnn_create(const float* host_params, int bf16, amg_cnn** out) {
  AMG_TRY
  if (!host_params || !out) fail(AMG_ERR_ARG, "NULL argument");
  check_params_finite(host_params, total_params());
  Cnn* N = new Cnn();
  try {
    N->bf16 = bf16 ? 1 : 0;
    for (int l = 0; l < NL; ++l) {
      N->nW[l] = (long)CH[l + 1] * CH[l] * 9;
      N->nB[l] = CH[l + 1];
      N->W32[l].ensure(sizeof(float) * N->nW[l]);
      N->B32[l].ensure(sizeof(float) * N->nB[l]);
      N->Ws[l].ensure(N->ssz() * N->nW[l]);
      for (Buf* b : {&N->mW[l], &N->vW[l], &N->gW[l]}) {
        b->ensure(sizeof(float) * N->nW[l]);
        HIPC(hipMemset(b->p, 0, sizeof(float) * N->nW[l]));
      }
      for (Buf* b : {&N->mB[l], &N->vB[l], &N->gB[l]}) {
        b->ensure(sizeof(float) * N->nB[l]);
        HIPC(hipMemset(b->p, 0, sizeof(float) * N->nB[l]));
      }
    }
    N->loss.ensure(sizeof(double));
    HIPC(hipHostMalloc((void**)&N->loss_host, sizeof(double), hipHostMallocDefault));
    upload_params(*N, host_params);
  } catch (...) {
    delete N;
    throw;
  }
  *out = N;
  AMG_CATCH
}

amg_status amg_cnn_destroy(amg_cnn* N) {
  AMG_TRY
  delete N;
  AMG_CATCH
}

amg_status amg_cnn_get_params(const amg_cnn* N, float* host_out) {
  AMG_TRY
  if (!N || !host_out) fail(AMG_ERR_ARG, "NULL argument");
  long off = 0;
  for (int l = 0; l < NL; ++l) {
    HIPC(hipMemcpy(host_out + off, N->W32[l].p, sizeof(float) * N->nW[l], hipMemcpyDeviceToHost));
    off += N->nW[l];
    HIPC(hipMemcpy(host_out + off, N->B32[l].p, sizeof(float) * N->nB[l], hipMemcpyDeviceToHost));
    off += N->nB[l];
  }
  AMG_CATCH
}

amg_status amg_cnn_set_params(amg_cnn* N, const float* host_params) {
  AMG_TRY
  if (!N || !host_params) fail(AMG_ERR_ARG, "NULL argument");
  check_params_finite(host_params, total_params());
  upload_params(*N, host_params);
  AMG_CATCH
}

amg_status amg_cnn_loss_grad(amg_cnn* N, const void* dev_links, const void* dev_vecs, int B, int L1, int L2,
                             double* loss, float* host_grads, void* stream) {
  AMG_TRY
  if (!N || !dev_links || !dev_vecs) fail(AMG_ERR_ARG, "NULL argument");
  check_lattice(B, L1, L2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cnn_ensure(*N, B, L2, L1);
  const bool g = host_grads != nullptr;
  const double L = N->bf16 ? loss_and_grads<bf16s>(*N, (const double2*)dev_links, (const double2*)dev_vecs, B, L2, L1, g, st)
                           : loss_and_grads<float>(*N, (const double2*)dev_links, (const double2*)dev_vecs, B, L2, L1, g, st);
  if (loss) *loss = L;
  if (g) {
    long off = 0;
    for (int l = 0; l < NL; ++l) {
      HIPC(hipMemcpy(host_grads + off, N->gW[l].p, sizeof(float) * N->nW[l], hipMemcpyDeviceToHost));
      off += N->nW[l];
      HIPC(hipMemcpy(host_grads + off, N->gB[l].p, sizeof(float) * N->nB[l], hipMemcpyDeviceToHost));
      off += N->nB[l];
    }
  }
  AMG_CATCH
}

amg_status amg_cnn_train_step(amg_cnn* N, const void* dev_links, const void* dev_vecs, int B, int L1, int L2,
                              float lr, double* loss, void* stream) {
  AMG_TRY
  if (!N || !dev_links || !dev_vecs) fail(AMG_ERR_ARG, "NULL argument");
  if (!(lr > 0.f) || !std::isfinite(lr)) fail(AMG_ERR_ARG, "learning rate must be positive");
  check_lattice(B, L1, L2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cnn_ensure(*N, B, L2, L1);
  const double L = N->bf16 ? loss_and_grads<bf16s>(*N, (const double2*)dev_links, (const double2*)dev_vecs, B, L2, L1, true, st)
                           : loss_and_grads<float>(*N, (const double2*)dev_links, (const double2*)dev_vecs, B, L2, L1, true, st);
  if (!std::isfinite(L)) fail(AMG_ERR_NAN, "non-finite loss; parameters not updated");
  N->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)N->step), c2 = 1.f - std::pow(b2, (float)N->step);
  for (int l = 0; l < NL; ++l) {
    hipLaunchKernelGGL(adam_kernel, dim3(nb(N->nW[l])), dim3(256), 0, st, N->W32[l].as<float>(), N->gW[l].as<float>(),
                       N->mW[l].as<float>(), N->vW[l].as<float>(), N->nW[l], lr, b1, b2, 1e-8f, c1, c2, N->Ws[l].p,
                       N->bf16);
    hipLaunchKernelGGL(adam_kernel, dim3(nb(N->nB[l])), dim3(256), 0, st, N->B32[l].as<float>(), N->gB[l].as<float>(),
                       N->mB[l].as<float>(), N->vB[l].as<float>(), N->nB[l], lr, b1, b2, 1e-8f, c1, c2, nullptr, 0);
  }
  HIPC(hipGetLastError());
  if (loss) *loss = L;
  AMG_CATCH
}

amg_status amg_cnn_propose(amg_cnn* N, const void* dev_links, int L1, int L2, void* dev_vecs_out, void* stream) {
  AMG_TRY
  if (!N || !dev_links || !dev_vecs_out) fail(AMG_ERR_ARG, "NULL argument");
  check_lattice(1, L1, L2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cnn_ensure(*N, 1, L2, L1);
  const long HW = (long)L1 * L2;
  const double2* U = (const double2*)dev_links;
  if (N->bf16) {
    forward<bf16s>(*N, U, 1, L2, L1, st);
    hipLaunchKernelGGL(proposals_kernel<bf16s>, dim3(nb(NVEC * HW)), dim3(256), 0, st, N->act[NL].as<bf16s>(),
                       N->phi.as<double>(), (double2*)dev_vecs_out, HW);
  } else {
    forward<float>(*N, U, 1, L2, L1, st);
    hipLaunchKernelGGL(proposals_kernel<float>, dim3(nb(NVEC * HW)), dim3(256), 0, st, N->act[NL].as<float>(),
                       N->phi.as<double>(), (double2*)dev_vecs_out, HW);
  }
  HIPC(hipGetLastError());
  AMG_CATCH
}

amg_status amg_cnn_forward(amg_cnn* N, const void* dev_links, int B, int L1, int L2, float* dev_out, void* stream) {
  AMG_TRY
  if (!N || !dev_links || !dev_out) fail(AMG_ERR_ARG, "NULL argument");
  check_lattice(B, L1, L2);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  cnn_ensure(*N, B, L2, L1);
  const long n = (long)B * 4 * NVEC * L1 * L2;
  if (N->bf16) {
    forward<bf16s>(*N, (const double2*)dev_links, B, L2, L1, st);
    hipLaunchKernelGGL(widen_kernel, dim3(nb(n)), dim3(256), 0, st, N->act[NL].as<bf16s>(), dev_out, n);
  } else {
    forward<float>(*N, (const double2*)dev_links, B, L2, L1, st);
    HIPC(hipMemcpyAsync(dev_out, N->act[NL].p, sizeof(float) * n, hipMemcpyDeviceToDevice, st));
  }
  HIPC(hipGetLastError());
  AMG_CATCH
}

}  // extern "C"

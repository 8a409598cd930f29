// 3-D CNN of the learned warm start and mass (include/cnn.h) on gfx950 MFMA.
//
// Every 3x3x3 convolution is an implicit GEMM on 16x16x16 bf16 MFMA tiles
// (float32 accumulation): a wave owns 16 consecutive voxels (rows) and all
// 16 output channels (columns); the K loop runs over (tap, input channel).
// Activations are channels-last bfloat16 [V][4] (input, 3 channels + zero
// pad) or [V][16]; pre-activations float32 [V][16].
// Lane layout of the MFMA (lane l, element i): A[l % 16][4 (l / 16) + i],
// B[4 (l / 16) + i][l % 16], D[4 (l / 16) + i][l % 16].
//
// Backward: the input gradient is the same convolution of the output gradient
// with mirrored taps and transposed weights, fused with GELU'(z); the weight
// gradient runs the MFMA with K over voxels (A = activations gathered per tap,
// B = output gradient), one partial per wave, summed in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/cnn.h"

namespace cnnk {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCin[4] = {3, 16, 16, 16};
constexpr int kCout[4] = {16, 16, 16, 2};
constexpr int kWaves = 2048;  // weight-gradient partials (one per wave)

inline int off_w(int l) {
  int o = 0;
  for (int k = 0; k < l; ++k) o += 27 * kCin[k] * kCout[k] + kCout[k];
  return o;
}
inline int off_b(int l) { return off_w(l) + 27 * kCin[l] * kCout[l]; }
inline int n_params() { return off_w(4); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
// GELU(z) = z Phi(z) with the normal CDF written as Phi(z) = erfc(-z / sqrt 2) / 2,
// which keeps its relative accuracy in the lower tail (1 + erf(.) cancels there)
__device__ __forceinline__ float norm_cdf(float z) { return 0.5f * erfcf(-z * 0.70710678118654752f); }
__device__ __forceinline__ float gelu(float z) { return z * norm_cdf(z); }
__device__ __forceinline__ float gelu_grad(float z) {
  return norm_cdf(z) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// ------------------------------------------------------------------ kernels
// in3 float [3][V] -> bf16 [V][4] (4th channel zero)
__global__ void __launch_bounds__(256) k_input(long long nv, const float* __restrict__ in3,
                                               uint16_t* __restrict__ a0) {
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long long)gridDim.x * 256) {
    ushort4 o;
    o.x = f2bf(in3[v]);
    o.y = f2bf(in3[nv + v]);
    o.z = f2bf(in3[2 * nv + v]);
    o.w = 0;
    reinterpret_cast<ushort4*>(a0)[v] = o;
  }
}

__global__ void __launch_bounds__(256) k_features(long long nv, const float* __restrict__ beta,
                                                  float scale, const float* __restrict__ mask,
                                                  const float* __restrict__ sel,
                                                  float* __restrict__ out3) {
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long long)gridDim.x * 256) {
    out3[v] = beta[v] * scale;
    out3[nv + v] = mask[v];
    out3[2 * nv + v] = sel[v];
  }
}

enum ConvMode : int { C_FWD_GELU = 0, C_FWD_LAST = 1, C_DGRAD = 2 };

// One wave per 16-voxel tile; CS = channel stride of the input (4 or 16),
// NC = K chunks (7 for the 3-channel input: 4 taps x 4 channels per chunk; 27
// otherwise).  The chunk loop is unrolled so that every gather of a tile is
// issued before the first MFMA needs it.  STORE_Z: keep the pre-activation for
// the backward pass (inference skips it).
template <int CS, int MODE, int NC, bool STORE_Z>
__global__ void __launch_bounds__(256) k_conv(int n, const uint16_t* __restrict__ in,
                                              const bf16x4* __restrict__ wp,
                                              const float* __restrict__ bias,
                                              const float* __restrict__ zprev,
                                              float* __restrict__ zout,
                                              uint16_t* __restrict__ aout) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long nv = (long long)n * n * n;
  const long long tile = (long long)blockIdx.x * 4 + wave;
  if (tile * 16 >= nv) return;  // no barriers below
  const int m = lane & 15, grp = lane >> 4;
  const long long v = tile * 16 + m;
  const int x = (int)(v / ((long long)n * n)), y = (int)((v / n) % n), z = (int)(v % n);
  bf16x4 a[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int tap = CS == 16 ? c : 4 * c + grp;
    const int ch0 = CS == 16 ? 4 * grp : 0;
    a[c] = bf16x4{0, 0, 0, 0};
    if (tap < 27) {
      const int xx = x + tap / 9 - 1, yy = y + (tap / 3) % 3 - 1, zz = z + tap % 3 - 1;
      if ((unsigned)xx < (unsigned)n && (unsigned)yy < (unsigned)n && (unsigned)zz < (unsigned)n)
        a[c] = *reinterpret_cast<const bf16x4*>(in + (((long long)xx * n + yy) * n + zz) * CS + ch0);
    }
  }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < NC; ++c)
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[c], wp[c * 64 + lane], acc, 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const long long vo = tile * 16 + 4 * grp + i;
    float val = acc[i];
    if (MODE == C_FWD_GELU) {
      val += bias[m];
      if (STORE_Z) zout[vo * 16 + m] = val;
      aout[vo * 16 + m] = f2bf(gelu(val));
    } else if (MODE == C_FWD_LAST) {
      zout[vo * 16 + m] = val + bias[m];
    } else {
      aout[vo * 16 + m] = f2bf(val * gelu_grad(zprev[vo * 16 + m]));
    }
  }
}

// 16-channel layers with the input brick staged in LDS: a block computes a
// brick of BX x BY x 16 voxels (x, y, z), loading it once with a one-voxel halo;
// each of its 4 waves takes BX * BY / 4 rows of 16 z-voxels (one MFMA tile each)
// and reads the 27 shifted A fragments from LDS.  Needs n a multiple of 16.
constexpr int kBX = 2, kBY = 8, kBZ = 16;
constexpr int kHX = kBX + 2, kHY = kBY + 2, kHZ = kBZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;  // voxels of the haloed brick
template <int MODE, bool STORE_Z>
__global__ void __launch_bounds__(256) k_conv_lds(int n, const uint16_t* __restrict__ in,
                                                  const bf16x4* __restrict__ wp,
                                                  const float* __restrict__ bias,
                                                  const float* __restrict__ zprev,
                                                  float* __restrict__ zout,
                                                  uint16_t* __restrict__ aout) {
  __shared__ uint4 brick[kHalo * 2];  // [voxel][2 x 8 bf16 channels]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nbz = n / kBZ, nby = n / kBY;
  const int bz = blockIdx.x % nbz, by = (blockIdx.x / nbz) % nby, bx = blockIdx.x / (nbz * nby);
  const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
  // stage the brick with its halo (zeros outside the grid)
  for (int i = threadIdx.x; i < kHalo * 2; i += 256) {
    const int vox = i >> 1, half = i & 1;
    const int hz = vox % kHZ, hy = (vox / kHZ) % kHY, hx = vox / (kHZ * kHY);
    const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
    uint4 val = make_uint4(0u, 0u, 0u, 0u);
    if ((unsigned)xx < (unsigned)n && (unsigned)yy < (unsigned)n && (unsigned)zz < (unsigned)n)
      val = reinterpret_cast<const uint4*>(in + (((long long)xx * n + yy) * n + zz) * 16)[half];
    brick[i] = val;
  }
  bf16x4 w[27];
#pragma unroll
  for (int c = 0; c < 27; ++c) w[c] = wp[c * 64 + lane];
  __syncthreads();
  const int m = lane & 15, grp = lane >> 4;
  const uint16_t* lb = reinterpret_cast<const uint16_t*>(brick);
  constexpr int kRows = kBX * kBY / 4;
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int row = wave * kRows + r;  // (x, y) row of the brick
    const int rx = row / kBY, ry = row % kBY;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 27; ++c) {
      const int hx = rx + c / 9, hy = ry + (c / 3) % 3, hz = m + c % 3;
      const bf16x4 a =
          *reinterpret_cast<const bf16x4*>(lb + ((hx * kHY + hy) * kHZ + hz) * 16 + 4 * grp);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w[c], acc, 0, 0, 0);
    }
    const long long vrow = ((long long)(x0 + rx) * n + (y0 + ry)) * n + z0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long vo = vrow + 4 * grp + i;
      float val = acc[i];
      if (MODE == C_FWD_GELU) {
        val += bias[m];
        if (STORE_Z) zout[vo * 16 + m] = val;
        aout[vo * 16 + m] = f2bf(gelu(val));
      } else if (MODE == C_FWD_LAST) {
        zout[vo * 16 + m] = val + bias[m];
      } else {
        aout[vo * 16 + m] = f2bf(val * gelu_grad(zprev[vo * 16 + m]));
      }
    }
  }
}

// mu, log-variance from the last layer's float32 output
__global__ void __launch_bounds__(256) k_outputs(long long nv, const float* __restrict__ z4,
                                                 float* __restrict__ mu, float* __restrict__ lv) {
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long long)gridDim.x * 256) {
    if (mu) mu[v] = z4[v * 16];
    if (lv) lv[v] = z4[v * 16 + 1];
  }
}

// Gaussian NLL per voxel; writes the bf16 output gradient [V][16] and block partials.
__global__ void __launch_bounds__(256) k_loss(long long nv, const float* __restrict__ z4,
                                              const float* __restrict__ target,
                                              uint16_t* __restrict__ dz4, double* __restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  const float inv = 1.f / (float)nv;
  for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nv; v += (long long)gridDim.x * 256) {
    const float mu = z4[v * 16], s = z4[v * 16 + 1];
    const float d = target[v] - mu, e = expf(-s);
    acc += 0.5 * ((double)d * d * e + s);
    uint16_t* o = dz4 + v * 16;
    o[0] = f2bf(-d * e * inv);
    o[1] = f2bf(0.5f * (1.f - d * d * e) * inv);
    for (int c = 2; c < 16; ++c) o[c] = 0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Weight gradient: dW[t][ci][co] = sum_v a[v + d_t][ci] dz[v][co]; one partial per wave.
template <int CS>
__global__ void __launch_bounds__(256) k_wgrad(int n, const uint16_t* __restrict__ a,
                                               const uint16_t* __restrict__ dz, int cpw,
                                               float* __restrict__ part, float* __restrict__ dbpart) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long nv = (long long)n * n * n;
  const long long nchunks = nv / 16;
  const int gw = blockIdx.x * 4 + wave;
  const int m = lane & 15, grp = lane >> 4;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;
  const long long c0 = (long long)gw * cpw;
  const long long c1 = c0 + cpw < nchunks ? c0 + cpw : nchunks;
  for (long long c = c0; c < c1; ++c) {
    int xs[4], ys[4], zs[4];
    bf16x4 b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long v = c * 16 + 4 * grp + i;
      xs[i] = (int)(v / ((long long)n * n));
      ys[i] = (int)((v / n) % n);
      zs[i] = (int)(v % n);
      const uint16_t g = dz[v * 16 + m];
      b[i] = (short)g;
      db += bf2f(g);
    }
#pragma unroll
    for (int t = 0; t < 27; ++t) {
      bf16x4 av = {0, 0, 0, 0};
      if (m < CS) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int xx = xs[i] + t / 9 - 1, yy = ys[i] + (t / 3) % 3 - 1, zz = zs[i] + t % 3 - 1;
          if ((unsigned)xx < (unsigned)n && (unsigned)yy < (unsigned)n && (unsigned)zz < (unsigned)n)
            av[i] = (short)a[(((long long)xx * n + yy) * n + zz) * CS + m];
        }
      }
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, acc[t], 0, 0, 0);
    }
  }
  float* o = part + (size_t)gw * 27 * 256;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) o[(t * 16 + 4 * grp + i) * 16 + m] = acc[t][i];
  db += __shfl_xor(db, 16);
  db += __shfl_xor(db, 32);
  if (lane < 16) dbpart[gw * 16 + lane] = db;
}

// Weight gradient with bricks staged in LDS, channel-major: the block walks
// bricks of BX x BY x 16 voxels; per brick it stages the haloed activations
// a[ci][voxel] and the output gradient dz[co][voxel], and each wave runs four
// K-steps (one 16-voxel z-row each) for all 27 taps, accumulating one partial
// per wave (A = shifted activations, rows ci; B = dz, columns co).
template <int CS>
__global__ void __launch_bounds__(256) k_wgrad_lds(int n, const uint16_t* __restrict__ a,
                                                   const uint16_t* __restrict__ dz,
                                                   float* __restrict__ part,
                                                   float* __restrict__ dbpart) {
  constexpr int kBV = kBX * kBY * kBZ;
  static_assert(kBV == 256 && kBX * kBY == 16, "one brick voxel per thread, four rows per wave");
  __shared__ uint16_t sa[CS][kHalo];
  __shared__ uint16_t sd[16][kBV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, grp = lane >> 4;
  const int nbz = n / kBZ, nby = n / kBY;
  const int nbricks = (n / kBX) * nby * nbz;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;
  for (int brick = blockIdx.x; brick < nbricks; brick += gridDim.x) {
    const int bz = brick % nbz, by = (brick / nbz) % nby, bx = brick / (nbz * nby);
    const int x0 = bx * kBX, y0 = by * kBY, z0 = bz * kBZ;
    __syncthreads();  // the previous brick's reads are done
    for (int vox = threadIdx.x; vox < kHalo; vox += 256) {
      const int hz = vox % kHZ, hy = (vox / kHZ) % kHY, hx = vox / (kHZ * kHY);
      const int xx = x0 + hx - 1, yy = y0 + hy - 1, zz = z0 + hz - 1;
      if ((unsigned)xx < (unsigned)n && (unsigned)yy < (unsigned)n && (unsigned)zz < (unsigned)n) {
        const uint16_t* src = a + (((long long)xx * n + yy) * n + zz) * CS;
#pragma unroll
        for (int ch = 0; ch < CS; ++ch) sa[ch][vox] = src[ch];
      } else {
#pragma unroll
        for (int ch = 0; ch < CS; ++ch) sa[ch][vox] = 0;
      }
    }
    {
      const int v = threadIdx.x;  // kBV == 256 voxels of the brick, one per thread
      const int vz = v % kBZ, vy = (v / kBZ) % kBY, vx = v / (kBZ * kBY);
      const uint4* src = reinterpret_cast<const uint4*>(
          dz + (((long long)(x0 + vx) * n + (y0 + vy)) * n + (z0 + vz)) * 16);
      const uint4 lo = src[0], hi = src[1];
      const uint32_t wds[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
      for (int ch = 0; ch < 16; ++ch)
        sd[ch][v] = (uint16_t)(ch & 1 ? wds[ch >> 1] >> 16 : wds[ch >> 1] & 0xffffu);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int row = wave * 4 + ks;  // (x, y) row of the brick, 16 voxels along z
      const int rx = row / kBY, ry = row % kBY;
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(&sd[m][row * kBZ + 4 * grp]);
#pragma unroll
      for (int i = 0; i < 4; ++i) db += bf2f((uint16_t)b[i]);
#pragma unroll
      for (int t = 0; t < 27; ++t) {
        const int hx = rx + t / 9, hy = ry + (t / 3) % 3, hz0 = 4 * grp + t % 3;
        bf16x4 av = {0, 0, 0, 0};
        if (m < CS) {
          const uint16_t* p = &sa[m < CS ? m : 0][(hx * kHY + hy) * kHZ + hz0];
#pragma unroll
          for (int i = 0; i < 4; ++i) av[i] = (short)p[i];
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, acc[t], 0, 0, 0);
      }
    }
  }
  const int gw = blockIdx.x * 4 + wave;
  float* o = part + (size_t)gw * 27 * 256;
#pragma unroll
  for (int t = 0; t < 27; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) o[(t * 16 + 4 * grp + i) * 16 + m] = acc[t][i];
  db += __shfl_xor(db, 16);
  db += __shfl_xor(db, 32);
  if (lane < 16) dbpart[gw * 16 + lane] = db;
}

// One layer's stored state in float32, [V][cout]: pre-activations (16-wide rows),
// bf16 activations and bf16 pre-activation gradients (either pointer may be null).
__global__ void __launch_bounds__(256) k_layer_state(long long nv, int cout,
                                                     const float* __restrict__ z16,
                                                     const uint16_t* __restrict__ a16,
                                                     const uint16_t* __restrict__ dz16,
                                                     float* __restrict__ z, float* __restrict__ a,
                                                     float* __restrict__ dz) {
  const long long tot = nv * cout;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < tot; i += (long long)gridDim.x * 256) {
    const long long v = i / cout, ch = i % cout;
    if (z) z[i] = z16[v * 16 + ch];
    if (a) a[i] = bf2f(a16[v * 16 + ch]);
    if (dz) dz[i] = bf2f(dz16[v * 16 + ch]);
  }
}

// Sum the per-wave partials of one layer into the flat gradient (fixed order).
__global__ void __launch_bounds__(256) k_wreduce(const float* __restrict__ part,
                                                 const float* __restrict__ dbpart, int nw, int cin,
                                                 int cout, float* __restrict__ gw, float* __restrict__ gb) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int nW = 27 * cin * cout;
  if (idx < nW) {
    const int t = idx / (cin * cout), ci = (idx / cout) % cin, co = idx % cout;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += part[((size_t)w * 27 + t) * 256 + ci * 16 + co];
    gw[idx] = s;
  } else if (idx < nW + cout) {
    const int co = idx - nW;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += dbpart[w * 16 + co];
    gb[co] = s;
  }
}

__global__ void __launch_bounds__(256) k_adam(int np, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m1, float* __restrict__ m2, float lr,
                                              float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  m1[i] = 0.9f * m1[i] + 0.1f * gi;
  m2[i] = 0.999f * m2[i] + 0.001f * gi * gi;
  p[i] -= lr * (m1[i] / c1) / (sqrtf(m2[i] / c2) + 1e-8f);
}

// bf16 MFMA B operands of one layer: forward (wp) and mirrored/transposed (wd).
__global__ void __launch_bounds__(256) k_pack(const float* __restrict__ W, int cin, int cout,
                                              int forward, int nchunk, bf16x4* __restrict__ out) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nchunk * 64) return;
  const int c = idx / 64, lane = idx % 64;
  bf16x4 r;
  for (int i = 0; i < 4; ++i) {
    float w = 0.f;
    if (forward) {
      const int co = lane % 16;
      int tap, ci;
      if (cin == 3) {
        tap = 4 * c + lane / 16;
        ci = i;
      } else {
        tap = c;
        ci = 4 * (lane / 16) + i;
      }
      if (tap < 27 && ci < cin && co < cout) w = W[(tap * cin + ci) * cout + co];
    } else {
      const int co = 4 * (lane / 16) + i, ci = lane % 16, tap = 26 - c;
      if (co < cout && ci < cin) w = W[(tap * cin + ci) * cout + co];
    }
    r[i] = (short)f2bf(w);
  }
  out[idx] = r;
}

}  // namespace cnnk

using namespace cnnk;

struct cnn_ctx {
  hipStream_t stream = nullptr;
  std::string err;
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  bf16x4* wp[4] = {nullptr, nullptr, nullptr, nullptr};
  bf16x4* wd[4] = {nullptr, nullptr, nullptr, nullptr};
  int steps = 0;
  int n = 0;
  bool grad_valid = false;  // the stored pre-activations and gradients belong to the last
                            // cnn_gradient / cnn_train_step
  // activations for the current N
  uint16_t *a0 = nullptr, *a[3] = {nullptr, nullptr, nullptr};
  // bf16 gradient of the loss with respect to each layer's pre-activations, one
  // buffer per layer so that the last backward pass can be inspected
  uint16_t* dz[4] = {nullptr, nullptr, nullptr, nullptr};
  float *z[4] = {nullptr, nullptr, nullptr, nullptr};
  float *wpart = nullptr, *dbpart = nullptr;
  double *lpart = nullptr, *lpart_h = nullptr;
};

namespace {
thread_local std::string g_cerr;

hmc_status cfail(cnn_ctx* c, hmc_status st, const std::string& why) {
  if (c) c->err = why;
  g_cerr = why;
  return st;
}

#define CCHK(c, call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) return cfail(c, HMC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int nchunk_fwd(int l) { return l == 0 ? 7 : 27; }

hmc_status pack_all(cnn_ctx* c) {
  for (int l = 0; l < 4; ++l) {
    const int nc = nchunk_fwd(l);
    hipLaunchKernelGGL(k_pack, dim3((nc * 64 + 255) / 256), dim3(256), 0, c->stream,
                       c->p + off_w(l), kCin[l], kCout[l], 1, nc, c->wp[l]);
    if (l > 0)
      hipLaunchKernelGGL(k_pack, dim3((27 * 64 + 255) / 256), dim3(256), 0, c->stream,
                         c->p + off_w(l), kCin[l], kCout[l], 0, 27, c->wd[l]);
  }
  CCHK(c, hipGetLastError());
  return HMC_OK;
}

void free_acts(cnn_ctx* c) {
  (void)hipFree(c->a0);
  for (int i = 0; i < 3; ++i) (void)hipFree(c->a[i]);
  for (int i = 0; i < 4; ++i) (void)hipFree(c->z[i]);
  for (int i = 0; i < 4; ++i) (void)hipFree(c->dz[i]);
  c->a0 = nullptr;
  for (int i = 0; i < 4; ++i) c->dz[i] = nullptr;
  for (int i = 0; i < 3; ++i) c->a[i] = nullptr;
  for (int i = 0; i < 4; ++i) c->z[i] = nullptr;
  c->n = 0;
}

hmc_status ensure(cnn_ctx* c, int n) {
  if (n < 4 || n % 4 != 0 || n > 512) return cfail(c, HMC_EINVAL, "N must be a multiple of 4 in 4..512");
  if (c->n == n) return HMC_OK;
  free_acts(c);
  const size_t nv = (size_t)n * n * n;
  CCHK(c, hipMalloc(&c->a0, nv * 4 * sizeof(uint16_t)));
  for (int i = 0; i < 3; ++i) CCHK(c, hipMalloc(&c->a[i], nv * 16 * sizeof(uint16_t)));
  for (int i = 0; i < 4; ++i) CCHK(c, hipMalloc(&c->z[i], nv * 16 * sizeof(float)));
  for (int i = 0; i < 4; ++i) CCHK(c, hipMalloc(&c->dz[i], nv * 16 * sizeof(uint16_t)));
  c->n = n;
  return HMC_OK;
}

template <bool STORE_Z>
hmc_status forward_t(cnn_ctx* c, int n, const float* in3) {
  const long long nv = (long long)n * n * n;
  const int blocks = (int)((nv / 16 + 3) / 4);
  hipLaunchKernelGGL(k_input, dim3(4096), dim3(256), 0, c->stream, nv, in3, c->a0);
  hipLaunchKernelGGL((k_conv<4, C_FWD_GELU, 7, STORE_Z>), dim3(blocks), dim3(256), 0, c->stream,
                     n, c->a0, c->wp[0], c->p + off_b(0), nullptr, c->z[0], c->a[0]);
  const bool lds = n % kBZ == 0;
  const int lblocks = lds ? (n / kBX) * (n / kBY) * (n / kBZ) : 0;
  for (int l = 1; l < 3; ++l) {
    if (lds)
      hipLaunchKernelGGL((k_conv_lds<C_FWD_GELU, STORE_Z>), dim3(lblocks), dim3(256), 0,
                         c->stream, n, c->a[l - 1], c->wp[l], c->p + off_b(l), nullptr, c->z[l],
                         c->a[l]);
    else
      hipLaunchKernelGGL((k_conv<16, C_FWD_GELU, 27, STORE_Z>), dim3(blocks), dim3(256), 0,
                         c->stream, n, c->a[l - 1], c->wp[l], c->p + off_b(l), nullptr, c->z[l],
                         c->a[l]);
  }
  // last layer: bias padded to 16 channels through a small device copy
  if (lds)
    hipLaunchKernelGGL((k_conv_lds<C_FWD_LAST, true>), dim3(lblocks), dim3(256), 0, c->stream, n,
                       c->a[2], c->wp[3], c->g + n_params(), nullptr, c->z[3], nullptr);
  else
    hipLaunchKernelGGL((k_conv<16, C_FWD_LAST, 27, true>), dim3(blocks), dim3(256), 0, c->stream,
                       n, c->a[2], c->wp[3], c->g + n_params(), nullptr, c->z[3], nullptr);
  CCHK(c, hipGetLastError());
  return HMC_OK;
}
// forward for training (keeps the pre-activations) and for inference
hmc_status forward(cnn_ctx* c, int n, const float* in3) { return forward_t<true>(c, n, in3); }
hmc_status infer(cnn_ctx* c, int n, const float* in3) {
  c->grad_valid = false;  // overwrites the activations of the last gradient evaluation
  return forward_t<false>(c, n, in3);
}

hmc_status gradient(cnn_ctx* c, int n, const float* in3, const float* target, double* loss) {
  c->grad_valid = false;
  hmc_status st = forward(c, n, in3);
  if (st != HMC_OK) return st;
  const long long nv = (long long)n * n * n;
  const int blocks = (int)((nv / 16 + 3) / 4);
  hipLaunchKernelGGL(k_loss, dim3(1024), dim3(256), 0, c->stream, nv, c->z[3], target, c->dz[3],
                     c->lpart);
  const long long nchunks = nv / 16;
  const bool lds = n % kBZ == 0;
  const int nbricks = lds ? (n / kBX) * (n / kBY) * (n / kBZ) : 0;
  const int cpw = (int)((nchunks + kWaves - 1) / kWaves);
  const int gblocks = lds ? std::min(nbricks, kWaves / 4) : 0;
  const int nw = lds ? 4 * gblocks : (int)((nchunks + cpw - 1) / cpw);
  const int wblocks = (nw + 3) / 4;
  for (int l = 3; l >= 0; --l) {
    const uint16_t* ain = l == 0 ? c->a0 : c->a[l - 1];
    const uint16_t* dz = c->dz[l];
    if (lds && l == 0)
      hipLaunchKernelGGL(k_wgrad_lds<4>, dim3(gblocks), dim3(256), 0, c->stream, n, ain, dz,
                         c->wpart, c->dbpart);
    else if (lds)
      hipLaunchKernelGGL(k_wgrad_lds<16>, dim3(gblocks), dim3(256), 0, c->stream, n, ain, dz,
                         c->wpart, c->dbpart);
    else if (l == 0)
      hipLaunchKernelGGL(k_wgrad<4>, dim3(wblocks), dim3(256), 0, c->stream, n, ain, dz, cpw,
                         c->wpart, c->dbpart);
    else
      hipLaunchKernelGGL(k_wgrad<16>, dim3(wblocks), dim3(256), 0, c->stream, n, ain, dz, cpw,
                         c->wpart, c->dbpart);
    const int tot = 27 * kCin[l] * kCout[l] + kCout[l];
    hipLaunchKernelGGL(k_wreduce, dim3((tot + 255) / 256), dim3(256), 0, c->stream, c->wpart,
                       c->dbpart, nw, kCin[l], kCout[l], c->g + off_w(l), c->g + off_b(l));
    if (l > 0) {
      if (n % kBZ == 0)
        hipLaunchKernelGGL((k_conv_lds<C_DGRAD, true>), dim3((n / kBX) * (n / kBY) * (n / kBZ)),
                           dim3(256), 0, c->stream, n, dz, c->wd[l], nullptr, c->z[l - 1],
                           nullptr, c->dz[l - 1]);
      else
        hipLaunchKernelGGL((k_conv<16, C_DGRAD, 27, true>), dim3(blocks), dim3(256), 0,
                           c->stream, n, dz, c->wd[l], nullptr, c->z[l - 1], nullptr, c->dz[l - 1]);
    }
  }
  CCHK(c, hipGetLastError());
  CCHK(c, hipMemcpyAsync(c->lpart_h, c->lpart, 1024 * sizeof(double), hipMemcpyDeviceToHost,
                         c->stream));
  CCHK(c, hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int i = 0; i < 1024; ++i) s += c->lpart_h[i];
  if (loss) *loss = s / (double)nv;
  c->grad_valid = true;
  return HMC_OK;
}

}  // namespace

extern "C" {

size_t cnn_param_count(void) { return (size_t)n_params(); }

const char* cnn_last_error(const cnn_ctx* c) { return c ? c->err.c_str() : g_cerr.c_str(); }

void cnn_destroy(cnn_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_acts(c);
  (void)hipFree(c->p);
  (void)hipFree(c->g);
  (void)hipFree(c->m1);
  (void)hipFree(c->m2);
  for (int l = 0; l < 4; ++l) {
    (void)hipFree(c->wp[l]);
    (void)hipFree(c->wd[l]);
  }
  (void)hipFree(c->wpart);
  (void)hipFree(c->dbpart);
  (void)hipFree(c->lpart);
  if (c->lpart_h) (void)hipHostFree(c->lpart_h);
  delete c;
}

hmc_status cnn_create(const float* params, void* stream, cnn_ctx** out) {
  if (!out || !params) return cfail(nullptr, HMC_EINVAL, "null argument");
  cnn_ctx* c = new cnn_ctx();
  c->stream = (hipStream_t)stream;
  const int np = n_params();
  auto bail = [&](const char* what, hipError_t e) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    g_cerr = c->err;
    cnn_destroy(c);
    return HMC_EDEVICE;
  };
  hipError_t e;
  // g holds the gradient and, past its end, the last layer's bias padded to 16
  if ((e = hipMalloc(&c->p, np * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&c->g, (np + 16) * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&c->m1, np * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipMalloc(&c->m2, np * sizeof(float))) != hipSuccess) return bail("hipMalloc", e);
  for (int l = 0; l < 4; ++l) {
    if ((e = hipMalloc(&c->wp[l], nchunk_fwd(l) * 64 * sizeof(bf16x4))) != hipSuccess)
      return bail("hipMalloc", e);
    if ((e = hipMalloc(&c->wd[l], 27 * 64 * sizeof(bf16x4))) != hipSuccess) return bail("hipMalloc", e);
  }
  if ((e = hipMalloc(&c->wpart, (size_t)kWaves * 27 * 256 * sizeof(float))) != hipSuccess)
    return bail("hipMalloc", e);
  if ((e = hipMalloc(&c->dbpart, (size_t)kWaves * 16 * sizeof(float))) != hipSuccess)
    return bail("hipMalloc", e);
  if ((e = hipMalloc(&c->lpart, 1024 * sizeof(double))) != hipSuccess) return bail("hipMalloc", e);
  if ((e = hipHostMalloc((void**)&c->lpart_h, 1024 * sizeof(double), 0)) != hipSuccess)
    return bail("hipHostMalloc", e);
  std::vector<float> zeros(np + 16, 0.f);
  if ((e = hipMemcpy(c->p, params, np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return bail("upload", e);
  if ((e = hipMemcpy(c->m1, zeros.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->m2, zeros.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->g, zeros.data(), (np + 16) * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return bail("upload", e);
  // padded last-layer bias after the gradient
  if ((e = hipMemcpy(c->g + np, params + off_b(3), 2 * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
    return bail("upload", e);
  if (pack_all(c) != HMC_OK) {
    g_cerr = c->err;
    cnn_destroy(c);
    return HMC_EDEVICE;
  }
  *out = c;
  return HMC_OK;
}

hmc_status cnn_get_params(cnn_ctx* c, float* params) {
  if (!c || !params) return cfail(c, HMC_EINVAL, "null argument");
  CCHK(c, hipMemcpyAsync(params, c->p, n_params() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  CCHK(c, hipStreamSynchronize(c->stream));
  return HMC_OK;
}

hmc_status cnn_forward(cnn_ctx* c, int32_t n, const float* in3, float* mu, float* logvar) {
  if (!c || !in3) return cfail(c, HMC_EINVAL, "null argument");
  hmc_status st = ensure(c, n);
  if (st != HMC_OK) return st;
  if ((st = infer(c, n, in3)) != HMC_OK) return st;
  const long long nv = (long long)n * n * n;
  hipLaunchKernelGGL(k_outputs, dim3(4096), dim3(256), 0, c->stream, nv, c->z[3], mu, logvar);
  CCHK(c, hipGetLastError());
  return HMC_OK;
}

hmc_status cnn_features(cnn_ctx* c, int32_t n, const float* beta, float beta_scale,
                        const float* mask, const float* sel, float* out3) {
  if (!c || !beta || !mask || !sel || !out3 || n < 4) return cfail(c, HMC_EINVAL, "bad argument");
  const long long nv = (long long)n * n * n;
  hipLaunchKernelGGL(k_features, dim3(4096), dim3(256), 0, c->stream, nv, beta, beta_scale, mask,
                     sel, out3);
  CCHK(c, hipGetLastError());
  return HMC_OK;
}

hmc_status cnn_gradient(cnn_ctx* c, int32_t n, const float* in3, const float* target, float* grad,
                        double* loss) {
  if (!c || !in3 || !target) return cfail(c, HMC_EINVAL, "null argument");
  hmc_status st = ensure(c, n);
  if (st != HMC_OK) return st;
  if ((st = gradient(c, n, in3, target, loss)) != HMC_OK) return st;
  if (grad) {
    CCHK(c, hipMemcpyAsync(grad, c->g, n_params() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    CCHK(c, hipStreamSynchronize(c->stream));
  }
  return HMC_OK;
}

hmc_status cnn_layer_state(cnn_ctx* c, int32_t layer, float* z, float* a, float* dz) {
  if (!c || layer < 0 || layer > 3 || (layer == 3 && a)) return cfail(c, HMC_EINVAL, "bad argument");
  if (c->n == 0 || !c->grad_valid) return cfail(c, HMC_EINVAL, "no cnn_gradient or cnn_train_step yet");
  const long long nv = (long long)c->n * c->n * c->n;
  hipLaunchKernelGGL(k_layer_state, dim3(4096), dim3(256), 0, c->stream, nv, kCout[layer],
                     c->z[layer], layer < 3 ? c->a[layer] : nullptr, c->dz[layer], z, a, dz);
  CCHK(c, hipGetLastError());
  return HMC_OK;
}

hmc_status cnn_train_step(cnn_ctx* c, int32_t n, const float* in3, const float* target, float lr,
                          double* loss) {
  if (!c || !in3 || !target || !(lr > 0)) return cfail(c, HMC_EINVAL, "bad argument");
  hmc_status st = ensure(c, n);
  if (st != HMC_OK) return st;
  if ((st = gradient(c, n, in3, target, loss)) != HMC_OK) return st;
  c->steps += 1;
  const float c1 = 1.f - std::pow(0.9f, (float)c->steps), c2 = 1.f - std::pow(0.999f, (float)c->steps);
  const int np = n_params();
  hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, c->stream, np, c->p, c->g, c->m1,
                     c->m2, lr, c1, c2);
  // keep the padded last-layer bias in step with the master copy
  CCHK(c, hipMemcpyAsync(c->g + np, c->p + off_b(3), 2 * sizeof(float), hipMemcpyDeviceToDevice,
                         c->stream));
  return pack_all(c);
}

}  // extern "C"

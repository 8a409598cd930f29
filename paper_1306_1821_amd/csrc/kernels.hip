// HIP kernels for the HMC density sampler (gfx950).
//
// One leapfrog step (kick-drift-kick, Sec. "The HMC algorithm") is four
// in-place passes over one intermediate half-complex grid T:
//   x-pass  (k space): forward x-FFT of the incoming gradient partial transform,
//           kick p_hat -= eps' (delta_hat / lambda_k + g_hat) (eq. HAMILTON2_a),
//           drift delta_hat += eps p_hat / m_k (eq. HAMILTON1_a), inverse x-FFT
//           of delta_hat -> T;
//   y-pass  inverse y-FFT;
//   z-pass  (real space): C2R along z gives delta, g = alpha delta - beta (the
//           data force of eq. Wiener_Posterior_force), R2C along z;
//   y-pass  forward y-FFT.
// alpha_i = sum_l b_l^2 Nbar_l R^l_i and beta_i = sum_l b_l (N^l_i - Nbar_l R^l_i)
// are precomputed once per sweep.  The unitary normalisation N^(-3/2) is
// applied in the x-pass (both directions).
#include <mutex>
#include <type_traits>

#include "hmc.h"
#include "kernels.hpp"
#include "fft.hpp"
#include "rng.hpp"
#include "samplers.hpp"

#ifndef HMC_NT
#define HMC_NT 1
#endif
// non-temporal hints on the state in the k-space pass (HMC_XNT) and on alpha,
// beta in the real-space pass (HMC_NT)
#ifndef HMC_ZWAVE
#define HMC_ZWAVE 1
#endif
#ifndef HMC_DOT_F32
#define HMC_DOT_F32 0
#endif
#ifndef HMC_LDS_TAB
#define HMC_LDS_TAB 1
#endif
#ifndef HMC_SHELL_LUT
#define HMC_SHELL_LUT 0
#endif
#ifndef HMC_ZPAD
#define HMC_ZPAD 1
#endif
#ifndef HMC_ZPRE
#define HMC_ZPRE 1
#endif
#ifndef HMC_XNT
#define HMC_XNT 0
#endif
// 256^3 pencil shapes (threads per pencil T, pencils per block B, radices):
// HMC_XCFG256 for the x and y passes, HMC_ZCFG256 for the z pass (measured
// alternatives kept selectable at build time)
#ifndef HMC_XCFG256
#define HMC_XCFG256 0
#endif
#ifndef HMC_ZCFG256
#define HMC_ZCFG256 1
#endif
#ifndef HMC_XCD
#define HMC_XCD 1
#endif
// z pass: padded LDS rows for the transform exchanges (HMC_ZLPAD) and the
// real-transform partner exchange X_k <-> X_{M-k} by DPP lane moves inside the
// row's lanes instead of an LDS round trip (HMC_ZDPP)
#ifndef HMC_ZLPAD
#define HMC_ZLPAD 1
#endif
#ifndef HMC_ZDPP
#define HMC_ZDPP 1
#endif
// twiddles of the single-size real-space pass read from LDS (HMC_ZTWL): their
// reads then leave the in-order vector-memory counter to the data loads, so the
// alpha, beta prefetch stays in flight through the first transform, and they are
// not held in registers across the tile loop
#ifndef HMC_ZTWL
#define HMC_ZTWL 1
#endif

namespace hmc {
using namespace hmcfft;

// Global-memory accesses.  Device pointers taken from the chain descriptor are
// generic to the compiler, which then emits flat instructions (counted by both
// the vector-memory and the LDS wait counters, so waits serialise); the casts to
// the global address space give global loads and stores.  The streamed state
// (delta_hat, p_hat, alpha, beta) carries the non-temporal hint (HMC_NT) so that
// it does not displace the intermediate grid from the caches.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) f2v gf2v;
typedef __attribute__((address_space(1))) const signed char gschar;
__device__ __forceinline__ float2 gld(const float2* p) {
  const f2v v = *(const gf2v*)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(float2* p, float2 v) {
  f2v w;
  w.x = v.x;
  w.y = v.y;
  *(gf2v*)p = w;
}
__device__ __forceinline__ float2 ld_s(const float2* p) {
#if HMC_NT
  const f2v v = __builtin_nontemporal_load((const gf2v*)p);
  return make_float2(v.x, v.y);
#else
  return gld(p);
#endif
}
__device__ __forceinline__ void st_s(float2* p, float2 v) {
#if HMC_NT
  f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (gf2v*)p);
#else
  gst(p, v);
#endif
}
// uniform base + 32-bit element offset: the byte offset is formed in 32 bits (every
// array of one chain is below 4 GiB), which lets the compiler use the
// scalar-base + 32-bit vector-offset form instead of a 64-bit address per element
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ float2 gldi(const float2* base, uint32_t i) {
  const f2v v = *(const gf2v*)((const gchar*)base + i * 8u);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gsti(float2* base, uint32_t i, float2 v) {
  f2v w;
  w.x = v.x;
  w.y = v.y;
  *(gf2v*)((gchar*)base + i * 8u) = w;
}
__device__ __forceinline__ float2 ld_si(const float2* base, uint32_t i) {
#if HMC_NT
  const f2v v = __builtin_nontemporal_load((const gf2v*)((const gchar*)base + i * 8u));
  return make_float2(v.x, v.y);
#else
  return gldi(base, i);
#endif
}
__device__ __forceinline__ void st_si(float2* base, uint32_t i, float2 v) {
#if HMC_NT
  f2v w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, (gf2v*)((gchar*)base + i * 8u));
#else
  gsti(base, i, v);
#endif
}
__device__ __forceinline__ float gldf(const float* p) {
  return *(const __attribute__((address_space(1))) float*)p;
}
__device__ __forceinline__ double gldd(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}
__device__ __forceinline__ float2 xld(const float2* base, uint32_t i) {
#if HMC_XNT
  return ld_si(base, i);
#else
  return gldi(base, i);
#endif
}
__device__ __forceinline__ void xst(float2* base, uint32_t i, float2 v) {
#if HMC_XNT
  st_si(base, i, v);
#else
  gsti(base, i, v);
#endif
}
// shell of a mode from the chain's q -> shell table (q = |k|^2 in grid units)
__device__ __forceinline__ int shell_lut(const signed char* lut, int q) {
  return (int)*(gschar*)(lut + q);
}

// ------------------------------------------------------------------ configs
// strided C2C passes (x and y): T threads per pencil, B pencils per block
template <int N> struct XC;
template <> struct XC<8>   { static constexpr int T = 2,  B = 128; using RL = Radices<4, 2>; };
template <> struct XC<16>  { static constexpr int T = 4,  B = 64;  using RL = Radices<4, 4>; };
template <> struct XC<32>  { static constexpr int T = 4,  B = 64;  using RL = Radices<8, 4>; };
template <> struct XC<64>  { static constexpr int T = 8,  B = 32;  using RL = Radices<8, 8>; };
// 128^3 x/y pencil shape: 16 threads x 16 columns, radices 8.4.4 (520 tiles; the
// 8 x 32 shape leaves 260 workgroups for 256 compute units: 5 % slower sweeps)
#ifndef HMC_XCFG128
#define HMC_XCFG128 1
#endif
#if HMC_XCFG128 == 1
template <> struct XC<128> { static constexpr int T = 16, B = 16;  using RL = Radices<8, 4, 4>; };
#elif HMC_XCFG128 == 2
template <> struct XC<128> { static constexpr int T = 32, B = 8;   using RL = Radices<4, 4, 4, 2>; };
#else
template <> struct XC<128> { static constexpr int T = 8,  B = 32;  using RL = Radices<16, 8>; };
#endif
template <> struct XC<192> { static constexpr int T = 16, B = 16;  using RL = Radices<4, 4, 12>; };
#if HMC_XCFG256 == 1
template <> struct XC<256> { static constexpr int T = 32, B = 8;   using RL = Radices<8, 8, 4>; };
#elif HMC_XCFG256 == 2
template <> struct XC<256> { static constexpr int T = 64, B = 4;   using RL = Radices<4, 4, 4, 4>; };
#else
template <> struct XC<256> { static constexpr int T = 16, B = 16;  using RL = Radices<16, 16>; };
#endif
// z pass: half-length complex transform of M = N/2 points per row
template <int N> struct ZC;
template <> struct ZC<8>   { static constexpr int T = 1, B = 256; using RL = Radices<4>; };
template <> struct ZC<16>  { static constexpr int T = 2, B = 128; using RL = Radices<4, 2>; };
template <> struct ZC<32>  { static constexpr int T = 4, B = 64;  using RL = Radices<4, 4>; };
template <> struct ZC<64>  { static constexpr int T = 4, B = 64;  using RL = Radices<8, 4>; };
template <> struct ZC<128> { static constexpr int T = 8, B = 32;  using RL = Radices<8, 8>; };
template <> struct ZC<192> { static constexpr int T = 8, B = 32;  using RL = Radices<4, 4, 6>; };
#if HMC_ZCFG256 == 1
template <> struct ZC<256> { static constexpr int T = 16, B = 16; using RL = Radices<8, 4, 4>; };
#elif HMC_ZCFG256 == 2
template <> struct ZC<256> { static constexpr int T = 32, B = 8;  using RL = Radices<4, 4, 4, 2>; };
#else
template <> struct ZC<256> { static constexpr int T = 8, B = 32;  using RL = Radices<16, 8>; };
#endif

// Radix plans of the single-size step passes.  Every plan keeps the B pencils per
// workgroup, so tiles, LDS size and the memory access pattern are plan-independent;
// the transform's stage count and LDS exchanges differ.  Plan 0 is the shape's
// default list; grids of 64^3 and more have two alternative radix lists at the same
// T threads per pencil (plans 1, 2) and, at 64^3, 128^3 and 256^3, a tile shape with
// twice the threads per pencil and half the values per thread (plan 3: 512-thread
// workgroups, fewer registers per thread, one more exchange).  The autotuner times
// them all (hmc_autotune / hmc_set_plan); plans only reach the k-space step pass,
// the y passes and the real-space force pass (plan 3 is plan 0 there).

template <int N> constexpr bool has_plans() { return N == 64 || N == 128 || N == 192 || N == 256; }
template <int N, int P> struct XPlan { using RL = typename XC<N>::RL; };
// threads per pencil of a plan (the shape's own T except for the plan-3 shapes)
template <int N, int P> struct XShape { static constexpr int T = XC<N>::T; };
template <> struct XPlan<64, 3>  { using RL = Radices<4, 4, 4>; };
template <> struct XShape<64, 3> { static constexpr int T = 2 * XC<64>::T; };
#if HMC_XCFG128 == 1
template <> struct XPlan<128, 3>  { using RL = Radices<4, 4, 4, 2>; };
template <> struct XShape<128, 3> { static constexpr int T = 2 * XC<128>::T; };
#endif
#if HMC_XCFG256 == 0
template <> struct XPlan<256, 3>  { using RL = Radices<8, 8, 4>; };
template <> struct XShape<256, 3> { static constexpr int T = 2 * XC<256>::T; };
#endif
template <int N, int P> constexpr int xthreads() { return XShape<N, P>::T * XC<N>::B; }
template <> struct XPlan<64, 1>  { using RL = Radices<4, 4, 4>; };
template <> struct XPlan<64, 2>  { using RL = Radices<2, 4, 8>; };
#if HMC_XCFG128 == 1
template <> struct XPlan<128, 1> { using RL = Radices<4, 8, 4>; };
template <> struct XPlan<128, 2> { using RL = Radices<2, 8, 8>; };
#elif HMC_XCFG128 == 2
template <> struct XPlan<128, 1> { using RL = Radices<2, 4, 4, 4>; };
template <> struct XPlan<128, 2> { using RL = Radices<4, 2, 4, 4>; };
#else
template <> struct XPlan<128, 1> { using RL = Radices<8, 16>; };
template <> struct XPlan<128, 2> { using RL = Radices<4, 4, 8>; };
#endif
template <> struct XPlan<192, 1> { using RL = Radices<12, 4, 4>; };
template <> struct XPlan<192, 2> { using RL = Radices<4, 12, 4>; };
template <> struct XPlan<256, 1> { using RL = Radices<4, 4, 16>; };
template <> struct XPlan<256, 2> { using RL = Radices<8, 8, 4>; };
template <int N, int P> struct ZPlan { using RL = typename ZC<N>::RL; };
template <> struct ZPlan<64, 1>  { using RL = Radices<4, 8>; };
template <> struct ZPlan<64, 2>  { using RL = Radices<2, 4, 4>; };
template <> struct ZPlan<128, 1> { using RL = Radices<4, 4, 4>; };
template <> struct ZPlan<128, 2> { using RL = Radices<2, 4, 8>; };
template <> struct ZPlan<192, 1> { using RL = Radices<6, 4, 4>; };
template <> struct ZPlan<192, 2> { using RL = Radices<4, 6, 4>; };
template <> struct ZPlan<256, 1> { using RL = Radices<4, 4, 8>; };
template <> struct ZPlan<256, 2> { using RL = Radices<2, 8, 8>; };

template <int N> constexpr int xlds() { return N * (XC<N>::B + 1) * 8; }
// z-pass LDS row stride in float2: at least M + 2; for M >= 64 rounded up to
// 16 mod 32 so that the two rows a half-wave reads fall on disjoint LDS banks
template <int N> constexpr int zrs() {
  constexpr int M = N / 2;
  if constexpr (M < 64 || !HMC_ZPAD) {
    return M + 2;
  } else {
    return ((M + 2 + 15) / 32) * 32 + 16;
  }
}
template <int N> constexpr int zlds() { return ZC<N>::B * zrs<N>() * 8; }
static_assert(HMC_ZLPAD == 0 || HMC_ZWAVE != 0, "padded z rows need the wavefront-scope transform");
#define HMC_ZROW_FITS(NN) static_assert((NN / 2 - 1) + (NN / 2 - 1) / 16 < zrs<NN>(), "padded z row");
HMC_ZROW_FITS(8) HMC_ZROW_FITS(16) HMC_ZROW_FITS(32) HMC_ZROW_FITS(64) HMC_ZROW_FITS(128)
HMC_ZROW_FITS(192) HMC_ZROW_FITS(256)
#undef HMC_ZROW_FITS

// z pass: each row (T threads, T divides 64) lies inside one wavefront and owns its
// LDS row, so its exchanges need only wavefront-scope ordering (HMC_ZWAVE)
__device__ __forceinline__ void zsync() { lds_sync<HMC_ZWAVE != 0>(); }
template <int N, int T, int DIR, class RL>
__device__ __forceinline__ void zfft(float2* v, float2* lds, int t, bool active,
                                     const float2* __restrict__ tw) {
  static_assert(64 % T == 0, "a z-pass row must not straddle wavefronts");
#if HMC_ZWAVE
  fft_wave<N, T, DIR, HMC_ZLPAD ? 4 : 0>(v, lds, 1, t, active, tw, RL{});
#else
  fft<N, T, DIR>(v, lds, 1, t, active, tw, RL{});
#endif
}

// the same with every twiddle read directly from an LDS-staged table
template <int N, int T, int DIR, class RL>
__device__ __forceinline__ void zfft_dtw(float2* v, float2* lds, int t, bool active,
                                         const float2* __restrict__ tw) {
  static_assert(64 % T == 0 && HMC_ZWAVE, "a z-pass row must not straddle wavefronts");
  fft_wave_dtw<N, T, DIR, HMC_ZLPAD ? 4 : 0>(v, lds, 1, t, active, tw, RL{});
}

// Real-transform partner of a row held by T consecutive lanes (T divides 16, rows
// aligned to T lanes): lane t >= 1 receives `src` of lane T - t of its row, lane 0
// keeps `own`.  T = 16: DPP row_mirror, then row_shr:1 (whose lane 0 has no source
// and keeps the old value); T = 8: row_half_mirror, row_shr:1 and a select for the
// second half's lane 0; T = 4: quad_perm [0,3,2,1]; T <= 2: lane T - t is the lane
// itself.
template <int T>
__device__ __forceinline__ float row_partner(float own, float src, int t) {
  const int o = __float_as_int(own), v = __float_as_int(src);
  if constexpr (T == 16) {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);
    return __int_as_float(__builtin_amdgcn_update_dpp(o, m, 0x111, 0xf, 0xf, false));
  } else if constexpr (T == 8) {
    const int m = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);
    const int r = __builtin_amdgcn_update_dpp(o, m, 0x111, 0xf, 0xf, false);
    return t == 0 ? own : __int_as_float(r);
  } else if constexpr (T == 4) {
    const int r = __builtin_amdgcn_update_dpp(0, v, 0x6c, 0xf, 0xf, false);
    return t == 0 ? own : __int_as_float(r);
  } else {
    static_assert(T == 1 || T == 2, "row partner: T must divide 16");
    return t == 0 ? own : src;
  }
}
template <int T>
__device__ __forceinline__ float2 row_partner(float2 own, float2 src, int t) {
  return make_float2(row_partner<T>(own.x, src.x, t), row_partner<T>(own.y, src.y, t));
}

// Real transform of length N = 2M through a complex one of length M, row held
// cyclically by T threads (element k = t + T e).  C2R input step: from the
// half-complex X (xr[e] = X_{t+Te}, xr[E] = X_M) form
//   Z_k = (X_k + conj X_{M-k}) + i W_N^-k (X_k - conj X_{M-k}),
// dropping the imaginary parts of the self-conjugate X_0 and X_M.  X_{M-k} sits
// in lane T - t as element E-1-e (t >= 1) and in lane 0 itself as element E - e;
// fetched by DPP lane moves (HMC_ZDPP), else through the LDS row L.
template <int N, int T, int E>
__device__ __forceinline__ void c2r_pre(const float2* xr, float2* v, float2* L, int t,
                                        const float2* __restrict__ twN) {
  constexpr int M = N / 2;
  if constexpr (HMC_ZDPP) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = t + T * e;
      float2 xa = xr[e], xb = cconj(row_partner<T>(xr[E - e], xr[E - 1 - e], t));
      if (k == 0) {
        xa = make_float2(xr[0].x, 0.f);
        xb = make_float2(xr[E].x, 0.f);
      }
      const float2 s = cadd(xa, xb);
      const float2 r = cmul(cconj(twN[k]), csub(xa, xb));
      v[e] = make_float2(s.x - r.y, s.y + r.x);
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) L[t + T * e] = xr[e];
    if (t == 0) L[M] = xr[E];
    zsync();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = t + T * e;
      float2 xa = L[k], xb = cconj(L[M - k]);
      if (k == 0) {
        xa = make_float2(L[0].x, 0.f);
        xb = make_float2(L[M].x, 0.f);
      }
      const float2 s = cadd(xa, xb);
      const float2 r = cmul(cconj(twN[k]), csub(xa, xb));
      v[e] = make_float2(s.x - r.y, s.y + r.x);
    }
    zsync();
  }
}

// R2C output step from Z = the length-M transform held cyclically in v:
//   X_k = E_k + W_N^k O_k, E_k = (Z_k + conj Z_{M-k})/2, O_k = -i (Z_k - conj Z_{M-k})/2,
// X_M = Re Z_0 - Im Z_0; st(k, X_k) for k = 0..M (active rows only).  Z_{M-k}: lane
// T - t, element E-1-e (t >= 1); lane 0, element (E - e) mod E.
template <int N, int T, int E, class Store>
__device__ __forceinline__ void r2c_post(const float2* v, float2* L, int t, bool active,
                                         const float2* __restrict__ twN, Store st) {
  constexpr int M = N / 2;
  float2 zcv[E];
  if constexpr (HMC_ZDPP) {
#pragma unroll
    for (int e = 0; e < E; ++e) zcv[e] = cconj(row_partner<T>(v[(E - e) % E], v[E - 1 - e], t));
  } else {
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) L[t + T * e] = v[e];
    }
    zsync();
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = t + T * e;
        zcv[e] = cconj(L[k == 0 ? 0 : M - k]);
      }
    }
  }
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = t + T * e;
      const float2 zk = v[e], zc = zcv[e];
      const float2 ev = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      const float2 df = csub(zk, zc);
      const float2 od = make_float2(0.5f * df.y, -0.5f * df.x);
      st(k, cadd(ev, cmul(twN[k], od)));
    }
    if (t == 0) st(M, make_float2(v[0].x - v[0].y, 0.f));
  }
}

#define HMC_FOR_N(X) X(8) X(16) X(32) X(64) X(128) X(192) X(256)

bool supported_n(int n) {
  return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 192 || n == 256;
}
int xpass_lds_bytes(int n) {
#define C(NN) if (n == NN) return xlds<NN>();
  HMC_FOR_N(C)
#undef C
  return 0;
}
int zpass_lds_bytes(int n) {
#define C(NN) if (n == NN) return zlds<NN>();
  HMC_FOR_N(C)
#undef C
  return 0;
}
int xpass_tiles(int n) {
#define C(NN) if (n == NN) return (NN * (NN / 2 + 1) + XC<NN>::B - 1) / XC<NN>::B;
  HMC_FOR_N(C)
#undef C
  return 0;
}
int zpass_tiles(int n) {
#define C(NN) if (n == NN) return (NN * NN + ZC<NN>::B - 1) / ZC<NN>::B;
  HMC_FOR_N(C)
#undef C
  return 0;
}

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_chain(const ChainDev* ch, int nch, int tile, int cls) {
  int c = 0;
  while (c + 1 < nch && tile >= ch[c + 1].tb[cls]) ++c;
  return c;
}

__device__ __forceinline__ int sfreq(int k, int n) { return k <= n / 2 ? k : k - n; }

// Tile handled by block b of a grid of g blocks.  Workgroups are dealt to the
// 8 XCDs round-robin; with HMC_XCD, XCD x takes a contiguous run of tiles so
// that neighbouring tiles (which share cache lines at their edges) hit the
// same L2.
__device__ __forceinline__ int tile_of(int b, int g) {
#if HMC_XCD
  const int q = g >> 3, r = g & 7, x = b & 7, i = b >> 3;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
#else
  (void)g;
  return b;
#endif
}

// Tiles a workgroup processes.  A grid with one workgroup per tile takes the
// XCD-aware order of tile_of.  A smaller (persistent) grid that is a multiple of 8
// walks, on each XCD, that XCD's contiguous run of tiles (workgroups are dealt to
// the 8 XCDs round-robin), so neighbouring tiles still share an L2; any other grid
// strides over all tiles.
struct TileWalk {
  int cur, end, step;
};
__device__ __forceinline__ TileWalk tile_walk(int total) {
  const int g = gridDim.x, b = blockIdx.x;
#if HMC_XCD
  if (g == total) {
    const int t = tile_of(b, total);
    return {t, t + 1, 1};
  }
  if ((g & 7) == 0 && g < total) {
    const int q = total >> 3, r = total & 7, x = b & 7, i = b >> 3;
    const int lo = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return {lo + i, lo + q + (x < r ? 1 : 0), g >> 3};
  }
#endif
  return {b, total, g};
}

// Shell of a mode: the m with m^2 q_max < nb^2 q <= (m+1)^2 q_max,
// q = |k|^2 in grid units, q_max = 3 (n/2)^2; -1 for q = 0.  Evaluated once per
// q into the chain's table (k_shell_lut); the passes look it up.
__device__ __forceinline__ int shell_q(uint64_t q, int n, int nb) {
  if (q == 0) return -1;
  const uint64_t qmax = 3ull * (uint64_t)(n / 2) * (uint64_t)(n / 2);
  const uint64_t lhs = (uint64_t)nb * (uint64_t)nb * q;
  int t = (int)ceilf(sqrtf((float)lhs / (float)qmax));
  if (t < 1) t = 1;
  while ((uint64_t)t * (uint64_t)t * qmax < lhs) ++t;
  while (t > 1 && (uint64_t)(t - 1) * (uint64_t)(t - 1) * qmax >= lhs) --t;
  return t - 1;
}
// The same rule evaluated in 32-bit integers with one float square root (exact for
// N <= 256, nb <= 128: nb^2 q and (m+1)^2 q_max stay below 2^31); the square root
// lands within one of the answer and one integer comparison each way corrects it.
// Branch-free: the hardware square root (about 1 ulp) gives t within one of the
// exact ceiling; one integer comparison each way corrects it.  No divergent
// branches, so the compiler can issue the loads of every element up front.
__device__ __forceinline__ int shell_fast(uint32_t q, uint32_t qmax, float inv_qmax, uint32_t nb) {
  const uint32_t lhs = nb * nb * q;
  int t = (int)ceilf(__builtin_amdgcn_sqrtf((float)lhs * inv_qmax));
  t = t < 1 ? 1 : t;
  t += (uint32_t)(t * t) * qmax < lhs ? 1 : 0;
  t -= ((t > 1) & ((uint32_t)((t - 1) * (t - 1)) * qmax >= lhs)) ? 1 : 0;
  return q == 0 ? -1 : t - 1;
}
__device__ __forceinline__ int shell_of(const ChainDev& d, int fx, int fy, int fz) {
  return shell_lut(d.lut, fx * fx + fy * fy + fz * fz);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Block size of the elementwise passes whose per-element work is a short dependent
// chain (shell sums, coefficients, accept / reject copies): 16 waves per tile in flight.
constexpr int kWideThreads = 1024;

// Deterministic block sum (fixed butterfly tree per wave, fixed wave order).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}
template <int W>  // the same for blocks of W waves
__device__ __forceinline__ double block_sum_w(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < W; ++w) s += red[w];
  return s;
}

// Shell bins of the k-space dot pass in LDS: kBinCopies copies per wave,
// bins[(wave * kBinCopies + copy) * kBinStride + m].  Lanes of neighbouring
// columns and neighbouring x frequencies (mostly the same shell) add into
// different copies, which cuts the same-address serialisation of the LDS atomics;
// each copy is written by one wave only, in program order, so the per-tile sums
// (fixed order over waves and copies) are reproducible.  The odd row stride puts
// the copies of one shell on different banks.  HMC_DOT_F32: float bins (flushed
// to float64 per tile).
#if HMC_DOT_F32
typedef float bin_t;
#else
typedef double bin_t;
#endif
#ifndef HMC_OBSMASK
#define HMC_OBSMASK 1  // coefficient and moment passes skip groups outside the survey support
#endif
#ifndef HMC_DOT_COPIES
#define HMC_DOT_COPIES 2
#endif
constexpr int kBinCopies = HMC_DOT_COPIES;
static_assert(kBinCopies == 1 || kBinCopies == 2 || kBinCopies == 4, "bin copies per wave");
constexpr int kBinStride = kMaxBins + 1;
constexpr int kBinSlots = 4 * kBinCopies * kBinStride;
// copy of a lane: bit 0 = column parity, bit 1 = parity of the pencil's x row
// within the wave (lane = row B + column for B < 64; the two low column bits for B >= 64)
template <int B>
__device__ __forceinline__ int bin_copy() {
  const int lane = threadIdx.x & 63;
  constexpr int hb = B >= 64 ? 1 : (B == 32 ? 5 : B == 16 ? 4 : B == 8 ? 3 : B == 4 ? 2 : 1);
  return ((lane & 1) | (((lane >> hb) & 1) << 1)) & (kBinCopies - 1);
}
template <class B>
__device__ __forceinline__ void bins_zero(B* bins) {
  for (int i = threadIdx.x; i < kBinSlots; i += kThreads) bins[i] = (B)0;
  __syncthreads();
}
template <class B>
__device__ __forceinline__ void bins_flush(B* bins, double* dst, int nb, int stride) {
  __syncthreads();
  for (int m = threadIdx.x; m < nb; m += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4 * kBinCopies; ++i) s += (double)bins[i * kBinStride + m];
    dst[(size_t)m * stride] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ x pass
// Thread (t, b) of a block holds elements kx = t + T e (e < E) of mode column
// col = tile B + b (ky = col / H, kz = col % H).  Idle lanes of the last tile read
// column 0 (in bounds) and store nothing.  Every load of an element is issued
// before its first use so that one wait covers them.
// F = 1: the joint move's shell-dot launch (X_FWD with XF_SCALE | XF_DOT | XF_NOSTORE,
// nothing stored), compiled for those flags without the per-element flag branches
template <int N, int MODE, int P = 0, int F = 0>
__device__ __forceinline__ void xpass(const ChainDev& d, int lt, const XArgs a, const float2* __restrict__ twall,
                      float2* lds, double* red, bin_t* bins) {
  using C = XC<N>;
  using RL = typename XPlan<N, P>::RL;
  constexpr int T = XShape<N, P>::T, B = C::B, E = N / T, H = N / 2 + 1, ES = B + 1;
  constexpr int NT = T * B;  // threads of the workgroup
  static_assert(NT == kThreads || MODE == X_STEP, "other tile shapes only for the step pass");
  constexpr uint32_t stride = (uint32_t)N * H;
  const float2* tw = twall + tw_offset(N);
  const int tid = threadIdx.x, b = tid % B, t = tid / B;
  const int col = lt * B + b;
  const bool active = col < N * H;
  const uint32_t colc = active ? col : 0;
  const int ky = colc / H, kz = colc % H;
  const int fy = sfreq(ky, N);
  const int q0 = fy * fy + kz * kz;
  const double wz = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
  const float norm = d.norm;
  const float kick = a.kick * d.eps, drift = a.drift * d.eps;
  float2* const Tb = d.T;
  float2* const dkb = d.dk;
  float2* const pkb = d.pk;
  float2* const gkb = d.gk;
  const signed char* const lut = d.lut;
#if HMC_LDS_TAB
  // per-shell float tables of the chain in LDS (indexed gathers stay on chip)
  __shared__ float stf[4 * kMaxBins];
  for (int i = tid; i < 4 * kMaxBins; i += NT) stf[i] = (i % kMaxBins) < d.nb ? gldf(d.tf + i) : 0.f;
  __syncthreads();
  const float* const tf = stf;
#else
  const float* const tf = d.tf;
#endif
  const double* const td = d.td;
  float2* L = lds + b;
  float2 v[E];
  auto offs = [&](int e) { return colc + (uint32_t)(t + T * e) * stride; };
  constexpr uint32_t qmax = 3u * (N / 2) * (N / 2);
  const float inv_qmax = 1.f / (float)qmax;
  const uint32_t nbu = (uint32_t)d.nb;
  auto shell = [&](int e) {
    const int fx = sfreq(t + T * e, N);
#if HMC_SHELL_LUT
    (void)inv_qmax;
    (void)nbu;
    return shell_lut(lut, q0 + fx * fx);
#else
    (void)lut;
    return shell_fast((uint32_t)(q0 + fx * fx), qmax, inv_qmax, nbu);
#endif
  };

  static_assert(F == 0 || MODE == X_FWD, "flag instantiation of X_FWD only");
  const bool dot = (MODE == X_FWD) && (F == 1 || (a.flags & XF_DOT));
  if (dot) bins_zero(bins);

  if constexpr (MODE != X_INV) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = gldi(Tb, offs(e));
    fft<N, T, +1>(v, L, ES, t, active, tw, RL{});
  }

  double acc0 = 0.0, acc1 = 0.0;
  if constexpr (MODE == X_INV) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int me = shell(e);
      const float2 x = gldi(dkb, offs(e));
      float s = norm;
      if ((a.flags & XF_SCALE) && me >= 0) s *= tf[kTScale + me];
      if ((a.flags & XF_PRIOR) && me >= 0) s *= rsqrtf(tf[kTInvLam + me]);  // sqrt(lambda_m)
      v[e] = me < 0 ? make_float2(0.f, 0.f) : cscale(x, s);
    }
  } else if constexpr (MODE == X_FWD && F == 1) {
    // every delta_hat load issued together (idle lanes read column 0, in bounds)
    float2 xk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) xk[e] = gldi(dkb, offs(e));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int me = shell(e);
      const bool on = active && me >= 0;
      const float2 g = cscale(v[e], norm);
      const float sc = tf[kTScale + (me >= 0 ? me : 0)];
      const double val = on ? wz * ((double)(sc * xk[e].x) * g.x + (double)(sc * xk[e].y) * g.y) : 0.0;
      if (on) atomicAdd(&bins[((threadIdx.x >> 6) * kBinCopies + bin_copy<B>()) * kBinStride + me], (bin_t)val);
    }
  } else if constexpr (MODE == X_FWD) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int me = shell(e);
      const float2 g = me < 0 ? make_float2(0.f, 0.f) : cscale(v[e], norm);
      if (active && !(a.flags & XF_NOSTORE)) {
        float2* out = (a.flags & XF_OUT_DK)     ? d.dk
                      : (a.flags & XF_OUT_ALT)  ? d.bgk
                      : (a.flags & XF_OUT_SHAT) ? d.shat
                                                : d.gk;
        gsti(out, offs(e), g);
      }
      if (dot) {
        double val = 0.0;
        int mm = -1;
        if (active && me >= 0) {
          const float2 x = gldi(dkb, offs(e));
          const float s = (a.flags & XF_SCALE) ? tf[kTScale + me] : 1.f;
          val = wz * ((double)(s * x.x) * g.x + (double)(s * x.y) * g.y);
          mm = me;
        }
        if (mm >= 0)
          atomicAdd(&bins[((threadIdx.x >> 6) * kBinCopies + bin_copy<B>()) * kBinStride + mm], (bin_t)val);
      }
    }
  } else {
    // X_START, X_STEP, X_END: kick (and drift).  All loads of the elements are
    // issued before the first use.
    float2 dkv[E], pkv[E];
    int m[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      m[e] = shell(e);
      dkv[e] = xld(dkb, offs(e));
      pkv[e] = MODE == X_START ? gldi(gkb, offs(e)) : xld(pkb, offs(e));  // X_START: g_hat
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int me = m[e];
      const float il = me >= 0 ? tf[kTInvLam + me] : 0.f;
      const float im = me >= 0 ? tf[kTInvMass + me] : 0.f;
      float2 dk = dkv[e], pk, g;
      if constexpr (MODE == X_START) {
        // fresh momentum p_hat = sqrt(m_k) F w; gradient of the current state from memory
        const float sq = me >= 0 ? tf[kTSqrtMass + me] : 0.f;
        pk = cscale(v[e], norm * sq);
        g = pkv[e];
        if (active) {
          gsti(d.bdk, offs(e), dk);
          gsti(d.bgk, offs(e), g);
        }
        if (active && me >= 0) {
          acc0 += wz * ((double)pk.x * pk.x + (double)pk.y * pk.y) * gldd(td + kDInvMass + me);
          acc1 += wz * ((double)dk.x * dk.x + (double)dk.y * dk.y) * gldd(td + kDInvLam + me);
        }
      } else {
        g = cscale(v[e], norm);
        pk = pkv[e];
      }
      if (me >= 0) {
        pk.x -= kick * (dk.x * il + g.x);
        pk.y -= kick * (dk.y * il + g.y);
        if constexpr (MODE != X_END) {
          dk.x += drift * pk.x * im;
          dk.y += drift * pk.y * im;
        }
      } else {
        pk = make_float2(0.f, 0.f);
        dk = make_float2(0.f, 0.f);
      }
      if constexpr (MODE == X_END) {
        if (active && me >= 0) {
          acc0 += wz * ((double)pk.x * pk.x + (double)pk.y * pk.y) * gldd(td + kDInvMass + me);
          acc1 += wz * ((double)dk.x * dk.x + (double)dk.y * dk.y) * gldd(td + kDInvLam + me);
        }
        if (active) {
          gsti(pkb, offs(e), pk);
          gsti(gkb, offs(e), me < 0 ? make_float2(0.f, 0.f) : g);
        }
      } else {
        if (active) {
          xst(dkb, offs(e), dk);
          xst(pkb, offs(e), pk);
        }
        v[e] = cscale(dk, norm);
      }
    }
  }

  if constexpr (MODE == X_INV || MODE == X_START || MODE == X_STEP) {
    fft<N, T, -1>(v, L, ES, t, active, tw, RL{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) gsti(Tb, offs(e), v[e]);
    }
  }
  if constexpr (MODE == X_START || MODE == X_END) {
    const double s0 = block_sum(0.5 * acc0, red);
    const double s1 = block_sum(0.5 * acc1, red);
    if (threadIdx.x == 0) {
      d.part[kPartKin * d.maxtiles + lt] = s0;
      d.part[kPartPri * d.maxtiles + lt] = s1;
    }
  }
  if (dot) bins_flush(bins, d.shpart + lt, d.nb, d.maxtiles);
  __syncthreads();
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_xpass(const ChainDev* __restrict__ ch, int nch,
                                                     int total, XArgs a,
                                                     const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  bin_t* bins = nullptr;
  if constexpr (MODE == X_FWD) {
    __shared__ bin_t sbins[kBinSlots];
    bins = sbins;
  }
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileXY);
    const ChainDev& d = ch[c];
    const int lt = tile - d.tb[kTileXY];
    switch (d.n) {
#define C(NN) case NN: xpass<NN, MODE>(d, lt, a, tw, lds, red, bins); break;
      HMC_FOR_N(C)
#undef C
      default: break;
    }
  }
}

// single-size variant: every chain of the launch has this N (lower register use)
template <int N, int MODE, int P = 0, int F = 0>
__global__ void __launch_bounds__((xthreads<N, P>())) k_xpass_n(const ChainDev* __restrict__ ch, int nch,
                                                       int total, XArgs a,
                                                       const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  bin_t* bins = nullptr;
  if constexpr (MODE == X_FWD) {
    __shared__ bin_t sbins[kBinSlots];
    bins = sbins;
  }
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileXY);
    const ChainDev& d = ch[c];
    xpass<N, MODE, P, F>(d, tile - d.tb[kTileXY], a, tw, lds, red, bins);
  }
}

// ------------------------------------------------------------------ y pass
template <int N, int DIR, int P = 0>
__device__ __forceinline__ void ypass(const ChainDev& d, int lt, const float2* __restrict__ twall, float2* lds,
                                      int buf) {
  using C = XC<N>;
  using RL = typename XPlan<N, P>::RL;
  constexpr int T = XShape<N, P>::T, B = C::B, E = N / T, H = N / 2 + 1, ES = B + 1;
  const float2* tw = twall + tw_offset(N);
  const int tid = threadIdx.x, b = tid % B, t = tid / B;
  const int p = lt * B + b;
  const bool active = p < N * H;
  const uint32_t x = active ? p / H : 0, kz = active ? p % H : 0;
  float2* const base = buf == 0 ? d.T : buf == 1 ? d.T2 : d.T3;
  const uint32_t o0 = x * (uint32_t)(N * H) + kz;  // idle lanes: column 0
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = gldi(base, o0 + (uint32_t)((t + T * e) * H));
  fft<N, T, DIR>(v, lds + b, ES, t, active, tw, RL{});
  if (active) {
#pragma unroll
    for (int e = 0; e < E; ++e) gsti(base, o0 + (uint32_t)((t + T * e) * H), v[e]);
  }
}

template <int DIR>
__global__ void __launch_bounds__(kThreads) k_ypass(const ChainDev* __restrict__ ch, int nch,
                                                     int total, const float2* __restrict__ tw,
                                                     int buf) {
  extern __shared__ float2 lds[];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileXY);
    const ChainDev& d = ch[c];
    const int lt = tile - d.tb[kTileXY];
    switch (d.n) {
#define C(NN) case NN: ypass<NN, DIR>(d, lt, tw, lds, buf); break;
      HMC_FOR_N(C)
#undef C
      default: break;
    }
  }
}

template <int N, int DIR, int P = 0>
__global__ void __launch_bounds__((xthreads<N, P>())) k_ypass_n(const ChainDev* __restrict__ ch, int nch,
                                                       int total, const float2* __restrict__ tw,
                                                       int buf) {
  extern __shared__ float2 lds[];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileXY);
    const ChainDev& d = ch[c];
    ypass<N, DIR, P>(d, tile - d.tb[kTileXY], tw, lds, buf);
  }
}

// ------------------------------------------------------------------ z pass
// twM: W_M^i (i < M), twN: W_N^k (k < M), in global memory or staged in LDS
template <int N, int MODE, int P = 0>
__device__ __forceinline__ void zpass_t(const ChainDev& d, int lt, const ZArgs a, const float2* twM,
                                        const float2* twN, float2* lds, double* red) {
  using C = ZC<N>;
  using RL = typename ZPlan<N, P>::RL;
  constexpr int M = N / 2, T = C::T, B = C::B, E = M / T, H = M + 1, RS = zrs<N>();
  const int tid = threadIdx.x, t = tid % T, b = tid / T;
  const int row = lt * B + b;
  const bool active = row < N * N;
  float2* L = lds + b * RS;
  const uint32_t rowc = active ? row : 0;  // idle lanes: row 0, nothing stored
  float2* const Tb = d.T;
  const uint32_t xo = rowc * (uint32_t)H;      // row start in T (elements)
  const uint32_t ro = rowc * (uint32_t)(N / 2);  // row start in a real field (voxel pairs)
  const size_t rbase = (size_t)rowc * N;
  float2 v[E];
  double dat = 0.0;
  // alpha, beta of the row (voxel pairs), loaded up front with the row of T;
  // idle lanes read row 0 and store nothing
  const bool data = MODE == Z_GRAD || (MODE == Z_C2R && (a.flags & ZF_DATA));
  constexpr bool pre = HMC_ZPRE && (MODE == Z_GRAD || MODE == Z_C2R);
  float2 al[pre ? E : 1], be[pre ? E : 1];
  if constexpr (pre) {
    if (data) {
      const float2* ap = reinterpret_cast<const float2*>(d.alpha);
      const float2* bp = reinterpret_cast<const float2*>(d.beta);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        al[e] = ld_si(ap, ro + t + T * e);
        be[e] = ld_si(bp, ro + t + T * e);
      }
    }
  }

  if constexpr (MODE == Z_GRAD || MODE == Z_C2R) {
    float2 xr[E + 1];
#pragma unroll
    for (int e = 0; e < E; ++e) xr[e] = gldi(Tb, xo + t + T * e);
    xr[E] = gldi(Tb, xo + M);
    c2r_pre<N, T, E>(xr, v, L, t, twN);
    zfft<M, T, -1, RL>(v, L, t, active, twM);
  } else if constexpr (MODE == Z_R2C) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = gldi(reinterpret_cast<const float2*>(a.src), ro + t + T * e);
  } else {  // Z_NOISE: white noise w_i from Philox stream 3 (11: warm start), element = voxel index
    const uint32_t stream = (a.flags & ZF_WARM) ? hmcrng::kWarm : hmcrng::kMomenta;
    if constexpr (T % 2 == 0 && E % 2 == 0) {
      // One Philox block covers 4 voxels: words 0, 1 go to the voxel pair of lane t
      // (t even) and words 2, 3 to that of lane t + 1.  For each element pair
      // (e, e + E/2) the even lane computes the block of e, the odd lane that of
      // e + E/2, and each hands its partner the two words the partner needs.
      const bool odd = t & 1;
#pragma unroll
      for (int e = 0; e < E / 2; ++e) {
        const uint64_t vox = rbase + 2 * (uint64_t)(t + T * (odd ? e + E / 2 : e));
        const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, stream, *d.draw, 0,
                                           (uint32_t)(vox >> 2));
        const uint32_t own0 = odd ? w.w[2] : w.w[0], own1 = odd ? w.w[3] : w.w[1];
        const uint32_t r0 = __shfl_xor(odd ? w.w[0] : w.w[2], 1);
        const uint32_t r1 = __shfl_xor(odd ? w.w[1] : w.w[3], 1);
        double z0, z1;
        hmcrng::box_muller(odd ? r0 : own0, odd ? r1 : own1, &z0, &z1);
        v[e] = make_float2((float)z0, (float)z1);
        hmcrng::box_muller(odd ? own0 : r0, odd ? own1 : r1, &z0, &z1);
        v[e + E / 2] = make_float2((float)z0, (float)z1);
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const uint64_t vox = rbase + 2 * (uint64_t)(t + T * e);
        const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, stream, *d.draw, 0,
                                           (uint32_t)(vox >> 2));
        double z0, z1;
        if (((vox >> 1) & 1) == 0)
          hmcrng::box_muller(w.w[0], w.w[1], &z0, &z1);
        else
          hmcrng::box_muller(w.w[2], w.w[3], &z0, &z1);
        v[e] = make_float2((float)z0, (float)z1);
      }
    }
  }

  if constexpr (MODE == Z_GRAD || MODE == Z_C2R) {
    float* drout = (a.flags & ZF_WRITE_DRN) ? d.drn : (a.flags & ZF_WRITE_DR) ? d.dr : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + T * e;
      const float2 x = v[e];
      if (active && drout) gsti(reinterpret_cast<float2*>(drout), ro + n, x);
      if (data) {
        float2 ae, bq;
        if constexpr (pre) {
          ae = al[e];
          bq = be[e];
        } else {
          ae = ld_si(reinterpret_cast<const float2*>(d.alpha), ro + n);
          bq = ld_si(reinterpret_cast<const float2*>(d.beta), ro + n);
        }
        if (active && (a.flags & ZF_DATA))
          dat += (0.5 * ae.x * x.x - bq.x) * (double)x.x + (0.5 * ae.y * x.y - bq.y) * (double)x.y;
        v[e] = make_float2(ae.x * x.x - bq.x, ae.y * x.y - bq.y);
      }
    }
  }

  if constexpr (MODE != Z_C2R) {
    zfft<M, T, +1, RL>(v, L, t, active, twM);
    r2c_post<N, T, E>(v, L, t, active, twN, [&](int k, float2 x) { gsti(Tb, xo + k, x); });
  }
  if (a.flags & ZF_DATA) {
    const double s = block_sum(dat, red);
    if (threadIdx.x == 0) d.part[kPartDat * d.maxtiles + lt] = s;
  }
  zsync();
}

template <int N, int MODE>
__device__ __forceinline__ void zpass(const ChainDev& d, int lt, const ZArgs a,
                                      const float2* __restrict__ twall, float2* lds, double* red) {
  zpass_t<N, MODE>(d, lt, a, twall + tw_offset(N / 2), twall + tw_offset(N), lds, red);
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_zpass(const ChainDev* __restrict__ ch, int nch,
                                                     int total, ZArgs a,
                                                     const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileZ);
    const ChainDev& d = ch[c];
    const int lt = tile - d.tb[kTileZ];
    switch (d.n) {
#define C(NN) case NN: zpass<NN, MODE>(d, lt, a, tw, lds, red); break;
      HMC_FOR_N(C)
#undef C
      default: break;
    }
  }
}

template <int N, int MODE, int P = 0>
__global__ void __launch_bounds__(kThreads) k_zpass_n(const ChainDev* __restrict__ ch, int nch,
                                                       int total, ZArgs a,
                                                       const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
#if HMC_ZTWL
  // the pass's twiddles staged in LDS once per workgroup: W_M^i, then W_N^k (k < M)
  __shared__ float2 stw[N];
  for (int i = threadIdx.x; i < N; i += kThreads)
    stw[i] = i < N / 2 ? tw[tw_offset(N / 2) + i] : tw[tw_offset(N) + i - N / 2];
  __syncthreads();
#endif
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const int c = find_chain(ch, nch, tile, kTileZ);
    const ChainDev& d = ch[c];
#if HMC_ZTWL
    zpass_t<N, MODE, P>(d, tile - d.tb[kTileZ], a, stw, stw + N / 2, lds, red);
#else
    zpass_t<N, MODE, P>(d, tile - d.tb[kTileZ], a, tw + tw_offset(N / 2), tw + tw_offset(N), lds, red);
#endif
  }
}


// ------------------------------------------------------------------ y-z plane pass
// One workgroup per real-space x plane of T (T holds the x pass's inverse x
// transform): inverse y transforms of the plane's kz columns, C2R along z, the
// data force g = alpha delta - beta, R2C along z and forward y transforms, with
// the plane on chip throughout.  It replaces the y, z, y pass sequence of a
// gradient evaluation, so the plane makes one round trip through HBM instead of
// three (T, alpha, beta read and T written once: 40 N^3 bytes per leapfrog step
// with the k-space pass instead of 56 N^3).
//
// The plane (N x (N/2+1) complex, 264 KB at 256^3) does not fit in LDS; it lives
// in the registers of a 512-thread workgroup (64 values per thread) and moves
// through LDS in chunks of rows for the column <-> row transposes.  The two
// self-conjugate columns kz = 0 and kz = M = N/2 travel as one complex column
// Z = C_0 + i C_M: both are Hermitian in ky (the field is real), so the inverse y
// transform of Z is y_0 + i y_M with y_0, y_M real, which are the real X_0, X_M
// every z row needs (the imaginary parts a C2R drops).  On the way back the real
// X_0, X_M of each row are packed the same way and separated after the forward y
// transform: A_k = (Z_k + conj Z_{-k}) / 2, B_k = -i (Z_k - conj Z_{-k}) / 2.
template <int N> struct PC;
template <> struct PC<256> {
  static constexpr int P = 512;          // threads per workgroup
  static constexpr int TY = 16;          // threads per y pencil (cyclic, 16 values each)
  using RLY = Radices<16, 16>;
  static constexpr int TZ = 16;          // threads per z row (cyclic, 8 values each)
  using RLZ = Radices<8, 4, 4>;          // the half-length (128-point) complex transform
  static constexpr int GL = 1;           // pencil groups that wait in LDS instead of registers
};
// 192^3: the plane (192 x 97 complex, 149 KB) in registers of 512 threads (36 values
// each, no group in LDS); radix-12 pencils, 8-thread z rows of the 96-point
// half-length transform (12 values each)
template <> struct PC<192> {
  static constexpr int P = 512;
  static constexpr int TY = 16;          // 12 values each
  using RLY = Radices<4, 4, 12>;
  static constexpr int TZ = 8;           // 12 values each
  using RLZ = Radices<4, 4, 6>;
  static constexpr int GL = 0;
};
// 64^3: the plane (64 x 33 complex, 17 KB) in registers of 256 threads (8 values
// each, one pencil group, one z chunk); 4-thread z rows of the 32-point transform
template <> struct PC<64> {
  static constexpr int P = 256;
  static constexpr int TY = 8;           // 8 values each
  using RLY = Radices<8, 8>;
  static constexpr int TZ = 4;           // 8 values each
  using RLZ = Radices<8, 4>;
  static constexpr int GL = 0;
};
// 128^3: the plane (128 x 65 complex, 66 KB) in registers of 512 threads (16 values
// each, no group in LDS); 8-thread z rows of the 64-point half-length transform
template <> struct PC<128> {
  static constexpr int P = 512;
  static constexpr int TY = 16;          // 8 values each
  using RLY = Radices<8, 4, 4>;
  static constexpr int TZ = 8;           // 8 values each
  using RLZ = Radices<8, 8>;
  static constexpr int GL = 0;
};
// LDS layout in float2: [0, A) the y-transform exchange and the z-row chunk buffer
// (used in turn), [A, A + N LS) the columns kept in LDS (row-major, stride LS),
// then N values for separating column 0
template <int N> struct PL {
  using C = PC<N>;
  static constexpr int M = N / 2, PY = C::P / C::TY, RZ = C::P / C::TZ;
  static constexpr int LY = N * (PY + 1), LZ = RZ * zrs<N>();
  static constexpr int A = LY > LZ ? LY : LZ;
  static constexpr int LS = C::GL * PY + 1;
  static constexpr int TOTAL = A + N * LS + N;
};

// compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1, so that
// register arrays indexed by I stay in registers however large the body is
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// FULL = false: the plain leapfrog step's launch (no data energy, no real field out),
// compiled without those branches (straight-line z-row code, no spilled registers)
template <int N, bool FULL>
__device__ __forceinline__ void yzpass(const ChainDev& d, int x, const ZArgs a, float2* lds,
                                       const float2* stw, double* red) {
  using C = PC<N>;
  using L = PL<N>;
  constexpr int M = N / 2, H = M + 1;
  constexpr int P = C::P, TY = C::TY, EY = N / TY, PY = P / TY, G = M / PY;
  constexpr int GL = C::GL, GR = G - GL, CR = GR * PY;  // register groups, their columns
  constexpr int TZ = C::TZ, EZ = M / TZ, RZ = P / TZ, NCH = N / RZ, EC = RZ / TY;
  constexpr int ESY = PY + 1, RSZ = zrs<N>(), LS = L::LS;
  static_assert(M % PY == 0 && N % RZ == 0 && RZ % TY == 0 && EY % EC == 0, "plane tiling");
  static_assert(64 % TZ == 0 && TZ <= 16, "a z row sits in one DPP row group of a wavefront");
  static_assert(CR % TZ == 0 && GR >= 1, "register / LDS column split on a row-thread boundary");
  // the plane's data energy goes to its own real-space tiles: a plane must cover whole
  // tiles of the real-space pass (at 32^3 and below one tile spans several planes)
  static_assert(N % ZC<N>::B == 0, "a plane covers whole real-space tiles");
  const int tid = threadIdx.x;
  const int b = tid % PY, t = tid / PY;   // column phase: pencil b of each group, its thread t
  const int r = tid / TZ, tz = tid % TZ;  // row phase: row r of the chunk, its thread tz
  // twiddles staged in LDS: W_M^i (i < M), W_N^k (k < M), then W_N^i (i < N) for the
  // y transforms (read from LDS, they are not kept in registers across the phases);
  // a transform stage reads the entries at powers of two of the radix index and forms
  // the others by complex products (fewer LDS reads than one read per twiddle)
  const float2* twM = stw;
  const float2* twN = stw + M;
  const float2* twy = stw + N;
  float2* const Ls = lds + L::A;          // columns CR .. M-1, [y][c - CR]
  // addresses: a uniform (scalar) base per element plus one per-thread offset, so
  // that the loads and stores of the plane share a single offset register
  float2* const Pl = d.T + (size_t)x * (N * H);
  const uint32_t toff = (uint32_t)(t * H + b);
  auto at = [&](int g, int e) {
    // the row base is pinned in scalar registers: left to itself the compiler folds
    // the constant into a 64-bit vector address per element and runs out of registers
    float2* p = Pl + TY * e * H;
    asm volatile("" : "+s"(p));
    return p + g * PY;
  };

  // the plane: packed column c = g PY + b, rows y = t + TY e (every load first);
  // groups below GR stay in registers, the others wait in LDS between the phases
  // column 0 of group 0 carries kz = 0 and kz = M: Z = C_0 + i C_M.  The kz = M
  // values are loaded first, so that waiting for them does not wait for the rest
  // of the plane (loads complete in order)
  float2 cm[EY];
  if (b == 0) {
#pragma unroll
    for (int e = 0; e < EY; ++e) cm[e] = gldi(at(0, e) + M, toff);
  }
  float2 v[GR][EY], u[GL > 0 ? GL : 1][EY];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int e = 0; e < EY; ++e) {
      const float2 val = gldi(at(g, e), toff);
      if (g < GR) v[g < GR ? g : 0][e] = val; else u[g < GR ? 0 : g - GR][e] = val;
    }
  if (b == 0) {
#pragma unroll
    for (int e = 0; e < EY; ++e) v[0][e] = make_float2(v[0][e].x - cm[e].y, v[0][e].y + cm[e].x);
  }
  static_for<0, G>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    if constexpr (g < GR) {
      fft<N, TY, -1>(v[g], lds + b, ESY, t, true, twy, typename C::RLY{});
    } else {
      fft<N, TY, -1>(u[g - GR], lds + b, ESY, t, true, twy, typename C::RLY{});
#pragma unroll
      for (int e = 0; e < EY; ++e) Ls[(t + TY * e) * LS + (g - GR) * PY + b] = u[g - GR][e];
    }
  });

  const float2* ap = reinterpret_cast<const float2*>(d.alpha);
  const float2* bp = reinterpret_cast<const float2*>(d.beta);
  float* drout = !FULL                      ? nullptr
                 : (a.flags & ZF_WRITE_DRN) ? d.drn
                 : (a.flags & ZF_WRITE_DR)  ? d.dr
                                            : nullptr;
  const bool data = FULL && (a.flags & ZF_DATA);
  float2* const Lr = lds + r * RSZ;  // this thread's row of the chunk buffer
  double dat = 0.0;
  // alpha and beta of chunk q + 1 are loaded as soon as chunk q's force is formed,
  // so that they arrive while chunk q finishes its transforms
  float2 al[EZ], be[EZ];
  auto load_ab = [&](int q) {
    const size_t rq = ((size_t)x * N + q * RZ) * M;  // the chunk's first voxel pair (uniform)
    const float2* ab = ap + rq;
    const float2* bb = bp + rq;
    asm volatile("" : "+s"(ab), "+s"(bb));  // scalar bases, one offset register (see at())
#pragma unroll
    for (int e = 0; e < EZ; ++e) {
      al[e] = ld_si(ab + TZ * e, (uint32_t)(r * M + tz));
      be[e] = ld_si(bb + TZ * e, (uint32_t)(r * M + tz));
    }
  };
  load_ab(0);
  static_for<0, NCH>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const size_t rq = ((size_t)x * N + q * RZ) * M;   // the chunk's first voxel pair (uniform)
    const uint32_t ro = (uint32_t)(r * M + tz);        // this thread's pair in the chunk
    float2* const Lsr = Ls + (q * RZ + r) * LS - CR;   // this row's columns CR.. in LDS
    __syncthreads();  // the buffer's previous readers are done
#pragma unroll
    for (int g = 0; g < GR; ++g)
#pragma unroll
      for (int j = 0; j < EC; ++j) lds[(t + TY * j) * RSZ + g * PY + b] = v[g][EC * q + j];
    __syncthreads();
    float2 xr[EZ + 1], w[EZ];
#pragma unroll
    for (int e = 0; e < EZ; ++e) {
      const int k = tz + TZ * e;
      xr[e] = TZ * e < CR ? Lr[k] : Lsr[k];
    }
    xr[EZ] = make_float2(xr[0].y, 0.f);  // lane 0: X_M from the packed column (X_0 = Re xr[0])
    c2r_pre<N, TZ, EZ>(xr, w, Lr, tz, twN);
    zfft<M, TZ, -1, typename C::RLZ>(w, Lr, tz, true, twM);
#pragma unroll
    for (int e = 0; e < EZ; ++e) {
      const float2 xv = w[e];
      if (FULL && drout) gsti(reinterpret_cast<float2*>(drout) + rq + TZ * e, ro, xv);  // trajectory ends
      if (data)
        dat += (0.5 * al[e].x * xv.x - be[e].x) * (double)xv.x +
               (0.5 * al[e].y * xv.y - be[e].y) * (double)xv.y;
      w[e] = make_float2(al[e].x * xv.x - be[e].x, al[e].y * xv.y - be[e].y);
    }
    if constexpr (q + 1 < NCH) load_ab(q + 1);
    zfft<M, TZ, +1, typename C::RLZ>(w, Lr, tz, true, twM);
    float x0 = 0.f;
    r2c_post<N, TZ, EZ>(w, Lr, tz, true, twN, [&](int k, float2 X) {
      if (k == 0)
        x0 = X.x;
      else if (k == M)
        Lr[0] = make_float2(x0, X.x);  // packed column 0: X_0 + i X_M
      else if (k < CR)
        Lr[k] = X;
      else
        Lsr[k] = X;
    });
    __syncthreads();
#pragma unroll
    for (int g = 0; g < GR; ++g)
#pragma unroll
      for (int j = 0; j < EC; ++j) v[g][EC * q + j] = lds[(t + TY * j) * RSZ + g * PY + b];
  });
  __syncthreads();
  // forward y transforms, each group stored as soon as it is done (the stores drain
  // while the next group transforms); column 0 of group 0 is separated first
  float2* const Lu = lds + (L::TOTAL - N);
  static_for<0, G>([&](auto gc) {
    constexpr int g = decltype(gc)::value;
    if constexpr (g < GR) {
      fft<N, TY, +1>(v[g], lds + b, ESY, t, true, twy, typename C::RLY{});
      if constexpr (g == 0) {
        // A_k = (Z_k + conj Z_-k) / 2 -> kz = 0, B_k = -i (Z_k - conj Z_-k) / 2 -> kz = M
        if (b == 0) {
#pragma unroll
          for (int e = 0; e < EY; ++e) Lu[t + TY * e] = v[0][e];
        }
        __syncthreads();
        if (b == 0) {
          float2 cb[EY];
#pragma unroll
          for (int e = 0; e < EY; ++e) {
            const int k = t + TY * e;
            const float2 z = v[0][e], zc = cconj(Lu[(N - k) % N]);  // N need not be a power of two
            const float2 df = csub(z, zc);
            v[0][e] = make_float2(0.5f * (z.x + zc.x), 0.5f * (z.y + zc.y));
            cb[e] = make_float2(0.5f * df.y, -0.5f * df.x);
          }
#pragma unroll
          for (int e = 0; e < EY; ++e) gsti(at(0, e) + M, toff, cb[e]);
        }
      }
#pragma unroll
      for (int e = 0; e < EY; ++e) gsti(at(g, e), toff, v[g][e]);
    } else {
#pragma unroll
      for (int e = 0; e < EY; ++e) u[g - GR][e] = Ls[(t + TY * e) * LS + (g - GR) * PY + b];
      fft<N, TY, +1>(u[g - GR], lds + b, ESY, t, true, twy, typename C::RLY{});
#pragma unroll
      for (int e = 0; e < EY; ++e) gsti(at(g, e), toff, u[g - GR][e]);
    }
  });
  if (data) {
    // the plane's data energy into the first of its z-pass tiles, zeros into the others
    constexpr int tpp = N / ZC<N>::B;
    const double sd = block_sum_w<P / 64>(dat, red);
    if (tid < tpp) d.part[kPartDat * d.maxtiles + x * tpp + tid] = tid == 0 ? sd : 0.0;
  }
}

// single-size launch: N consecutive workgroups per chain, one per x plane
template <int N, bool FULL>
__global__ void __launch_bounds__(PC<N>::P) k_yzpass_n(const ChainDev* __restrict__ ch, ZArgs a,
                                                        const float2* __restrict__ tw) {
  __shared__ float2 lds[PL<N>::TOTAL];
  __shared__ float2 stw[2 * N];
  __shared__ double red[PC<N>::P / 64];
  for (int i = threadIdx.x; i < 2 * N; i += PC<N>::P)
    stw[i] = i < N / 2 ? tw[tw_offset(N / 2) + i] : i < N ? tw[tw_offset(N) + i - N / 2] : tw[tw_offset(N) + i - N];
  __syncthreads();
  yzpass<N, FULL>(ch[blockIdx.x / N], (int)(blockIdx.x % N), a, lds, stw, red);
}

bool plane_pass_supported(int n) { return n == 64 || n == 128 || n == 192 || n == 256; }
template <int N>
static void launch_yz_n(const ChainDev* ch, int nch, ZArgs a, const float2* tw, hipStream_t s) {
  if (a.flags & (ZF_DATA | ZF_WRITE_DR | ZF_WRITE_DRN))
    hipLaunchKernelGGL((k_yzpass_n<N, true>), dim3(nch * N), dim3(PC<N>::P), 0, s, ch, a, tw);
  else
    hipLaunchKernelGGL((k_yzpass_n<N, false>), dim3(nch * N), dim3(PC<N>::P), 0, s, ch, a, tw);
}
void launch_yzpass(const ChainDev* ch, int nch, ZArgs a, const float2* tw, hipStream_t s, int n) {
  switch (n) {
    case 256: launch_yz_n<256>(ch, nch, a, tw, s); break;
    case 192: launch_yz_n<192>(ch, nch, a, tw, s); break;
    case 128: launch_yz_n<128>(ch, nch, a, tw, s); break;
    case 64: launch_yz_n<64>(ch, nch, a, tw, s); break;
    default: break;
  }
}

// ------------------------------------------------------------------ learned mass
// Inverse mass T T^T, T = P D^(1/2) F^-1 diag(m_k^-1/2) (P removes the mean):
//   drift  delta_hat += eps [F(D^(1/2) F^-1(p_hat / m_k))]_{k != 0}
//   kick   p_hat -= eps F(D^(1/2) P grad psi),
//          grad psi = F^-1(delta_hat / lambda) + alpha delta - beta;
// F(D^(1/2) P g) = F(D^(1/2) g) - mean(g) F(D^(1/2)), with mean(g) from the
// real-space pass partials and F(D^(1/2)) precomputed.  A step is
//   x L_DRIFT (T2 -> drift -> delta_hat, inverse x of delta_hat -> T and of
//   delta_hat/lambda -> T3), y-1 T, y-1 T3, z LZ_FORCE (T, T3 -> T), y+1 T,
//   x L_KICK (T -> kick -> inverse x of p_hat/m -> T2), y-1 T2, z LZ_VEL, y+1 T2.

// C2R of one half-complex row into v (v[e] = (x_2n, x_2n+1), n = t + T e).
template <int N>
__device__ __forceinline__ void row_c2r(const float2* X, float2* L, float2* v, int t, bool active,
                                        const float2* __restrict__ twN,
                                        const float2* __restrict__ twM) {
  using C = ZC<N>;
  constexpr int M = N / 2, T = C::T, E = M / T;
  float2 xr[E + 1];
#pragma unroll
  for (int e = 0; e < E; ++e) xr[e] = gld(X + t + T * e);  // X: an in-bounds row for idle lanes
  xr[E] = gld(X + M);
  c2r_pre<N, T, E>(xr, v, L, t, twN);
  zfft<M, T, -1, typename C::RL>(v, L, t, active, twM);
}

// R2C of v (same distribution) into the half-complex row X.
template <int N>
__device__ __forceinline__ void row_r2c(float2* v, float2* L, float2* X, int t, bool active,
                                        const float2* __restrict__ twN,
                                        const float2* __restrict__ twM) {
  using C = ZC<N>;
  constexpr int M = N / 2, T = C::T, E = M / T;
  zfft<M, T, +1, typename C::RL>(v, L, t, active, twM);
  r2c_post<N, T, E>(v, L, t, active, twN, [&](int k, float2 x) { gst(X + k, x); });
  zsync();
}

template <int N, int MODE>
__device__ __forceinline__ void zpass_l(const ChainDev& d, int lt, const ZArgs a,
                                        const float2* __restrict__ twall, float2* lds,
                                        double* red) {
  using C = ZC<N>;
  constexpr int M = N / 2, T = C::T, B = C::B, E = M / T, H = M + 1, RS = zrs<N>();
  const float2* twM = twall + tw_offset(M);
  const float2* twN = twall + tw_offset(N);
  const int tid = threadIdx.x, t = tid % T, b = tid / T;
  const int row = lt * B + b;
  const bool active = row < N * N;
  float2* L = lds + b * RS;
  const uint32_t rowc = active ? row : 0;  // idle lanes: row 0, nothing stored
  const uint32_t roff = rowc * (uint32_t)H;
  const uint32_t ro = rowc * (uint32_t)(N / 2);
  const float2* sm = reinterpret_cast<const float2*>(d.smass);
  float2 v[E], s[E];
#pragma unroll
  for (int e = 0; e < E; ++e) s[e] = gldi(sm, ro + t + T * e);
  double sum = 0.0, dat = 0.0;
  if constexpr (MODE == LZ_FORCE) {
    float2 al[E], be[E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      al[e] = ld_si(reinterpret_cast<const float2*>(d.alpha), ro + t + T * e);
      be[e] = ld_si(reinterpret_cast<const float2*>(d.beta), ro + t + T * e);
    }
    row_c2r<N>(d.T3 + roff, L, w, t, active, twN, twM);  // prior force F^-1(delta_hat/lambda)
    row_c2r<N>(d.T + roff, L, v, t, active, twN, twM);   // delta
    float* drout = (a.flags & ZF_WRITE_DRN) ? d.drn : (a.flags & ZF_WRITE_DR) ? d.dr : nullptr;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = t + T * e;
      const float2 x = v[e], fp = w[e];
      if (active && drout) gsti(reinterpret_cast<float2*>(drout), ro + n, x);
      const float g0 = fp.x + al[e].x * x.x - be[e].x, g1 = fp.y + al[e].y * x.y - be[e].y;
      if (active) {
        sum += (double)g0 + (double)g1;
        if (a.flags & ZF_DATA)
          dat += (0.5 * al[e].x * x.x - be[e].x) * (double)x.x +
                 (0.5 * al[e].y * x.y - be[e].y) * (double)x.y;
      }
      v[e] = make_float2(s[e].x * g0, s[e].y * g1);
    }
  } else {
    row_c2r<N>(d.T2 + roff, L, v, t, active, twN, twM);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = make_float2(s[e].x * v[e].x, s[e].y * v[e].y);
  }
  row_r2c<N>(v, L, (MODE == LZ_FORCE ? d.T : d.T2) + roff, t, active, twN, twM);
  if constexpr (MODE == LZ_FORCE) {
    const double s1 = block_sum(sum, red);
    if (threadIdx.x == 0) d.part[kPartAux * d.maxtiles + lt] = s1;
    if (a.flags & ZF_DATA) {
      const double s2 = block_sum(dat, red);
      if (threadIdx.x == 0) d.part[kPartDat * d.maxtiles + lt] = s2;
    }
  }
  zsync();
}

template <int N, int MODE>
__device__ __forceinline__ void xpass_l(const ChainDev& d, int lt, const XArgs a,
                                        const float2* __restrict__ twall, float2* lds,
                                        double* red) {
  using C = XC<N>;
  constexpr int T = C::T, B = C::B, E = N / T, H = N / 2 + 1, ES = B + 1;
  constexpr uint32_t stride = (uint32_t)N * H;
  const float2* tw = twall + tw_offset(N);
  const int tid = threadIdx.x, b = tid % B, t = tid / B;
  const int col = lt * B + b;
  const bool active = col < N * H;
  const uint32_t colc = active ? col : 0;  // idle lanes: column 0, nothing stored
  const int ky = colc / H, kz = colc % H;
  const int fy = sfreq(ky, N);
  const int q0 = fy * fy + kz * kz;
  const double wz = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
  const float norm = d.norm;
  const float kick = a.kick * d.eps, drift = a.drift * d.eps;
  constexpr bool KICK = MODE == L_KICK || MODE == L_KICK_LAST;
  __shared__ float stf[4 * kMaxBins];
  for (int i = tid; i < 4 * kMaxBins; i += kThreads) stf[i] = (i % kMaxBins) < d.nb ? gldf(d.tf + i) : 0.f;
  __syncthreads();
  const float* const tf = stf;
  const double* const td = d.td;
  constexpr uint32_t qmax = 3u * (N / 2) * (N / 2);
  const float inv_qmax = 1.f / (float)qmax;
  float2* L = lds + b;
  const float2* src = MODE == L_DRIFT ? d.T2 : d.T;
  auto offs = [&](int e) { return colc + (uint32_t)(t + T * e) * stride; };
  float2 v[E], w[E], sv[E];
  int m[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int fx = sfreq(t + T * e, N);
    m[e] = shell_fast((uint32_t)(q0 + fx * fx), qmax, inv_qmax, (uint32_t)d.nb);
    v[e] = gldi(src, offs(e));
    sv[e] = MODE == L_START || MODE == L_DRIFT ? xld(d.dk, offs(e)) : xld(d.pk, offs(e));
    w[e] = KICK ? gldi(d.shat, offs(e)) : MODE == L_START ? gldi(d.gk, offs(e))
                                                          : make_float2(0.f, 0.f);
  }
  fft<N, T, +1>(v, L, ES, t, active, tw, typename C::RL{});
  const float gbar = KICK ? (float)d.P[kGbar] : 0.f;
  double acc0 = 0.0, acc1 = 0.0;
  const float2 z2 = make_float2(0.f, 0.f);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int me = m[e];
    const float il = me >= 0 ? tf[kTInvLam + me] : 0.f;
    if constexpr (MODE == L_START) {
      const float sq = me >= 0 ? tf[kTSqrtMass + me] : 0.f;
      const float2 pk = cscale(v[e], norm * sq);
      const float2 dk = me >= 0 ? sv[e] : z2;
      if (active) {
        gsti(d.bdk, offs(e), dk);
        gsti(d.bgk, offs(e), w[e]);
        xst(d.pk, offs(e), pk);
        if (me >= 0) {
          acc0 += wz * ((double)pk.x * pk.x + (double)pk.y * pk.y) * gldd(td + kDInvMass + me);
          acc1 += wz * ((double)dk.x * dk.x + (double)dk.y * dk.y) * gldd(td + kDInvLam + me);
        }
      }
      v[e] = cscale(dk, norm);
      w[e] = cscale(dk, norm * il);
    } else if constexpr (MODE == L_DRIFT) {
      float2 dk = me >= 0 ? sv[e] : z2;
      if (me >= 0) {
        dk.x += drift * norm * v[e].x;
        dk.y += drift * norm * v[e].y;
      }
      if (active) xst(d.dk, offs(e), dk);
      v[e] = cscale(dk, norm);
      w[e] = cscale(dk, norm * il);
    } else {
      float2 pk = me >= 0 ? sv[e] : z2;
      if (me >= 0) {
        const float2 sh = w[e];
        pk.x -= kick * (norm * v[e].x - gbar * sh.x);
        pk.y -= kick * (norm * v[e].y - gbar * sh.y);
      }
      if (active) xst(d.pk, offs(e), pk);
      if constexpr (MODE == L_KICK_LAST) {
        if (active && me >= 0) {
          const float2 dk = xld(d.dk, offs(e));
          acc0 += wz * ((double)pk.x * pk.x + (double)pk.y * pk.y) * gldd(td + kDInvMass + me);
          acc1 += wz * ((double)dk.x * dk.x + (double)dk.y * dk.y) * gldd(td + kDInvLam + me);
        }
      } else {
        v[e] = me >= 0 ? cscale(pk, norm * tf[kTInvMass + me]) : z2;
      }
    }
  }
  if constexpr (MODE == L_START || MODE == L_DRIFT) {
    fft<N, T, -1>(v, L, ES, t, active, tw, typename C::RL{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) gsti(d.T, offs(e), v[e]);
    }
    fft<N, T, -1>(w, L, ES, t, active, tw, typename C::RL{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) gsti(d.T3, offs(e), w[e]);
    }
  } else if constexpr (MODE == L_KICK) {
    fft<N, T, -1>(v, L, ES, t, active, tw, typename C::RL{});
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) gsti(d.T2, offs(e), v[e]);
    }
  }
  if constexpr (MODE == L_START || MODE == L_KICK_LAST) {
    const double s0 = block_sum(0.5 * acc0, red);
    const double s1 = block_sum(0.5 * acc1, red);
    if (threadIdx.x == 0) {
      d.part[kPartKin * d.maxtiles + lt] = s0;
      d.part[kPartPri * d.maxtiles + lt] = s1;
    }
  }
  __syncthreads();
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_xpass_l(const ChainDev* __restrict__ ch, int nch,
                                                       int total, XArgs a,
                                                       const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileXY)];
    const int lt = tile - d.tb[kTileXY];
    switch (d.n) {
#define C(NN) case NN: xpass_l<NN, MODE>(d, lt, a, tw, lds, red); break;
      HMC_FOR_N(C)
#undef C
      default: break;
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(kThreads) k_zpass_l(const ChainDev* __restrict__ ch, int nch,
                                                       int total, ZArgs a,
                                                       const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const int tile = w.cur;
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileZ)];
    const int lt = tile - d.tb[kTileZ];
    switch (d.n) {
#define C(NN) case NN: zpass_l<NN, MODE>(d, lt, a, tw, lds, red); break;
      HMC_FOR_N(C)
#undef C
      default: break;
    }
  }
}

// single-size variants of the learned passes (every chain of the launch has this N)
template <int N, int MODE>
__global__ void __launch_bounds__(kThreads) k_xpass_l_n(const ChainDev* __restrict__ ch, int nch,
                                                         int total, XArgs a,
                                                         const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const ChainDev& d = ch[find_chain(ch, nch, w.cur, kTileXY)];
    xpass_l<N, MODE>(d, w.cur - d.tb[kTileXY], a, tw, lds, red);
  }
}
template <int N, int MODE>
__global__ void __launch_bounds__(kThreads) k_zpass_l_n(const ChainDev* __restrict__ ch, int nch,
                                                         int total, ZArgs a,
                                                         const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  __shared__ double red[4];
  for (TileWalk w = tile_walk(total); w.cur < w.end; w.cur += w.step) {
    const ChainDev& d = ch[find_chain(ch, nch, w.cur, kTileZ)];
    zpass_l<N, MODE>(d, w.cur - d.tb[kTileZ], a, tw, lds, red);
  }
}

// learned-mass factor: phase 0 sums exp(logvar) per tile, phase 1 writes
// D^(1/2) = sqrt(exp(logvar) / mean(exp(logvar)))
__global__ void __launch_bounds__(kThreads) k_mass_prep(const ChainDev* __restrict__ ch, int total,
                                                         const float* __restrict__ lv, int phase) {
  __shared__ double red[4];
  const ChainDev& d = ch[0];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
      const long long i = (long long)tile * kElemPerTile + j;
      if (i >= d.nv) break;
      if (phase == 0)
        acc += exp((double)lv[i]);
      else
        d.smass[i] = (float)sqrt(exp((double)lv[i]) / d.P[kLmean]);
    }
    if (phase == 0) {
      const double s = block_sum(acc, red);
      if (threadIdx.x == 0) d.part[kPartAux * d.maxtiles + tile] = s;
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_shell_lut(const ChainDev* __restrict__ ch) {
  const ChainDev& d = ch[0];
  const int qmax = 3 * (d.n / 2) * (d.n / 2);
  for (int q = blockIdx.x * kThreads + threadIdx.x; q <= qmax; q += gridDim.x * kThreads)
    d.lut[q] = (signed char)shell_q((uint64_t)q, d.n, d.nb);
}

// results of the last trajectory / sweep into caller device buffers (no host
// round trip): trajectories write dH and the accept flag per chain; sweeps write
// per chain the record [dH, accepted, rj_dH, rj_accepted, status, rj_wall_hits,
// P_m (physical units), b_l, Nbar_l], records back to back in chain order
__global__ void k_export(const ChainDev* __restrict__ ch, int nch, int sweep, double* rec,
                         int32_t* acc) {
  const int i = blockIdx.x;
  if (i >= nch) return;
  const ChainDev& d = ch[i];
  if (!sweep) {
    if (threadIdx.x == 0) {
      rec[i] = d.P[kDH];
      acc[i] = d.P[kAcc] != 0.0 ? 1 : 0;
    }
    return;
  }
  long long off = 0;
  for (int j = 0; j < i; ++j) off += kRecHead + ch[j].nb + 2 * ch[j].nsub;
  double* r = rec + off;
  const double f = d.box * d.box * d.box / ((double)d.n * d.n * d.n);
  if (threadIdx.x == 0) {
    r[0] = d.P[kDH];
    r[1] = d.P[kAcc];
    r[2] = d.P[kRjDH];
    r[3] = d.P[kRjAcc];
    r[4] = d.P[kStatus];
    r[5] = d.P[kRjHits];
  }
  for (int m = threadIdx.x; m < d.nb; m += blockDim.x) r[kRecHead + m] = d.P[kLam + m] * f;
  for (int l = threadIdx.x; l < d.nsub; l += blockDim.x) {
    r[kRecHead + d.nb + l] = d.P[kBias + l];
    r[kRecHead + d.nb + d.nsub + l] = d.P[kNbar + l];
  }
}

// warm start: drn <- mu + sqrt(v / sigma^2) drn with v = exp(logvar), drn the
// prior draw F^-1(sqrt(lambda_k) F w) and sigma^2 = (1/N^3) sum_m n_m lambda_m its
// per-voxel variance
__global__ void __launch_bounds__(kThreads) k_warm_combine(const ChainDev* __restrict__ ch,
                                                            int total, const float* __restrict__ mu,
                                                            const float* __restrict__ lv) {
  __shared__ double inv_s2;
  const ChainDev& d = ch[0];
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int m = 0; m < d.nb; ++m) s += d.P[kNmodes + m] * d.P[kLam + m];
    inv_s2 = (double)d.nv / s;
  }
  __syncthreads();
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
      const long long i = (long long)tile * kElemPerTile + j;
      if (i >= d.nv) break;
      d.drn[i] = (float)(mu[i] + sqrt(exp((double)lv[i]) * inv_s2) * d.drn[i]);
    }
  }
}

// ------------------------------------------------------------------ launches
static inline int grid_of(int total, int cap) { return total < cap || cap <= 0 ? total : cap; }

// plan: radix plan of the step pass (X_STEP), y passes and the force pass (Z_GRAD)
template <int N>
static void launch_x_n(int mode, dim3 g, dim3 bl, int lds, hipStream_t s, const ChainDev* ch,
                       int nch, int total, XArgs a, const float2* tw, int plan) {
  switch (mode) {
    case X_INV: hipLaunchKernelGGL((k_xpass_n<N, X_INV>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_FWD:
      if (a.flags == (XF_SCALE | XF_DOT | XF_NOSTORE))
        hipLaunchKernelGGL((k_xpass_n<N, X_FWD, 0, 1>), g, bl, lds, s, ch, nch, total, a, tw);
      else
        hipLaunchKernelGGL((k_xpass_n<N, X_FWD>), g, bl, lds, s, ch, nch, total, a, tw);
      break;
    case X_START: hipLaunchKernelGGL((k_xpass_n<N, X_START>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_STEP:
      if constexpr (has_plans<N>()) {
        if (plan == 1) {
          hipLaunchKernelGGL((k_xpass_n<N, X_STEP, 1>), g, bl, lds, s, ch, nch, total, a, tw);
          break;
        }
        if (plan == 2) {
          hipLaunchKernelGGL((k_xpass_n<N, X_STEP, 2>), g, bl, lds, s, ch, nch, total, a, tw);
          break;
        }
        if (plan == 3) {
          hipLaunchKernelGGL((k_xpass_n<N, X_STEP, 3>), g, dim3(xthreads<N, 3>()), lds, s, ch, nch,
                             total, a, tw);
          break;
        }
      }
      hipLaunchKernelGGL((k_xpass_n<N, X_STEP>), g, bl, lds, s, ch, nch, total, a, tw);
      break;
    case X_END: hipLaunchKernelGGL((k_xpass_n<N, X_END>), g, bl, lds, s, ch, nch, total, a, tw); break;
  }
}
template <int N, int DIR>
static void launch_y_n(dim3 g, dim3 bl, int lds, hipStream_t s, const ChainDev* ch, int nch,
                       int total, const float2* tw, int buf, int plan) {
  if constexpr (has_plans<N>()) {
    if (plan == 1) {
      hipLaunchKernelGGL((k_ypass_n<N, DIR, 1>), g, bl, lds, s, ch, nch, total, tw, buf);
      return;
    }
    if (plan == 2) {
      hipLaunchKernelGGL((k_ypass_n<N, DIR, 2>), g, bl, lds, s, ch, nch, total, tw, buf);
      return;
    }
    if (plan == 3) {
      hipLaunchKernelGGL((k_ypass_n<N, DIR, 3>), g, dim3(xthreads<N, 3>()), lds, s, ch, nch, total,
                         tw, buf);
      return;
    }
  }
  hipLaunchKernelGGL((k_ypass_n<N, DIR>), g, bl, lds, s, ch, nch, total, tw, buf);
}
template <int N>
static void launch_z_n(int mode, dim3 g, dim3 bl, int lds, hipStream_t s, const ChainDev* ch,
                       int nch, int total, ZArgs a, const float2* tw, int plan) {
  switch (mode) {
    case Z_GRAD:
      if constexpr (has_plans<N>()) {
        if (plan == 1) {
          hipLaunchKernelGGL((k_zpass_n<N, Z_GRAD, 1>), g, bl, lds, s, ch, nch, total, a, tw);
          break;
        }
        if (plan == 2) {
          hipLaunchKernelGGL((k_zpass_n<N, Z_GRAD, 2>), g, bl, lds, s, ch, nch, total, a, tw);
          break;
        }
      }
      hipLaunchKernelGGL((k_zpass_n<N, Z_GRAD>), g, bl, lds, s, ch, nch, total, a, tw);
      break;
    case Z_NOISE: hipLaunchKernelGGL((k_zpass_n<N, Z_NOISE>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case Z_C2R: hipLaunchKernelGGL((k_zpass_n<N, Z_C2R>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case Z_R2C: hipLaunchKernelGGL((k_zpass_n<N, Z_R2C>), g, bl, lds, s, ch, nch, total, a, tw); break;
  }
}

// uniform_n > 0: every chain of the launch has that N (single-size kernels);
// otherwise the mixed-size kernels dispatch per tile.
void launch_xpass(int mode, const ChainDev* ch, int nch, int total, int lds, XArgs a,
                  const float2* tw, int cap, hipStream_t s, int uniform_n, int plan) {
  dim3 g(grid_of(total, cap)), bl(kThreads);
  switch (uniform_n) {
#define C(NN) case NN: launch_x_n<NN>(mode, g, bl, lds, s, ch, nch, total, a, tw, plan); return;
    HMC_FOR_N(C)
#undef C
    default: break;
  }
  switch (mode) {
    case X_INV: hipLaunchKernelGGL(k_xpass<X_INV>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_FWD: hipLaunchKernelGGL(k_xpass<X_FWD>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_START: hipLaunchKernelGGL(k_xpass<X_START>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_STEP: hipLaunchKernelGGL(k_xpass<X_STEP>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case X_END: hipLaunchKernelGGL(k_xpass<X_END>, g, bl, lds, s, ch, nch, total, a, tw); break;
  }
}
void launch_ypass(int dir, const ChainDev* ch, int nch, int total, int lds, const float2* tw,
                  int cap, hipStream_t s, int uniform_n, int buf, int plan) {
  dim3 g(grid_of(total, cap)), bl(kThreads);
  switch (uniform_n) {
#define C(NN)                                                                  \
  case NN:                                                                     \
    if (dir > 0)                                                               \
      launch_y_n<NN, 1>(g, bl, lds, s, ch, nch, total, tw, buf, plan);         \
    else                                                                       \
      launch_y_n<NN, -1>(g, bl, lds, s, ch, nch, total, tw, buf, plan);        \
    return;
    HMC_FOR_N(C)
#undef C
    default: break;
  }
  if (dir > 0)
    hipLaunchKernelGGL(k_ypass<1>, g, bl, lds, s, ch, nch, total, tw, buf);
  else
    hipLaunchKernelGGL(k_ypass<-1>, g, bl, lds, s, ch, nch, total, tw, buf);
}
void launch_zpass(int mode, const ChainDev* ch, int nch, int total, int lds, ZArgs a,
                  const float2* tw, int cap, hipStream_t s, int uniform_n, int plan) {
  dim3 g(grid_of(total, cap)), bl(kThreads);
  switch (uniform_n) {
#define C(NN) case NN: launch_z_n<NN>(mode, g, bl, lds, s, ch, nch, total, a, tw, plan); return;
    HMC_FOR_N(C)
#undef C
    default: break;
  }
  switch (mode) {
    case Z_GRAD: hipLaunchKernelGGL(k_zpass<Z_GRAD>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case Z_NOISE: hipLaunchKernelGGL(k_zpass<Z_NOISE>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case Z_C2R: hipLaunchKernelGGL(k_zpass<Z_C2R>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case Z_R2C: hipLaunchKernelGGL(k_zpass<Z_R2C>, g, bl, lds, s, ch, nch, total, a, tw); break;
  }
}

// ------------------------------------------------------------------ elementwise
// Real-space tiles cover kElemPerTile voxels; k-space tiles kElemPerTile modes.

// alpha, beta from R, counts, bias, Nbar (voxels with R > 0 only); partial sum of alpha.
// real fields are read 4 voxels at a time (N^3 and the tile size are multiples of 4)
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f4v gf4v;
__device__ __forceinline__ f4v gld4(const float* base, uint32_t i4) {
  return *(const gf4v*)((const gchar*)base + i4 * 16u);
}
__device__ __forceinline__ void gst4(float* base, uint32_t i4, f4v v) {
  *(gf4v*)((gchar*)base + i4 * 16u) = v;
}

// Survey support bitmask (once at init; R must not change afterwards).  A wave
// covers 64 consecutive 4-voxel groups starting at a multiple of 64 (tiles hold
// 4096 groups, N^3 / 4 is a multiple of 64), so its ballot is one mask word.
__global__ void __launch_bounds__(kThreads) k_obs_mask(const ChainDev* __restrict__ ch, int nch,
                                                        int total) {
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    const uint32_t nv4 = (uint32_t)(d.nv / 4), base4 = (uint32_t)lt * (kElemPerTile / 4);
    for (uint32_t j = threadIdx.x; j < kElemPerTile / 4; j += kThreads) {
      const uint32_t i4 = base4 + j;
      if (i4 >= nv4) break;  // wave-uniform (see above)
      bool o = false;
      for (int l = 0; l < d.nsub; ++l) {
        const f4v r = gld4(d.R + (size_t)l * d.nv, i4);
        o |= (r[0] > 0.f) | (r[1] > 0.f) | (r[2] > 0.f) | (r[3] > 0.f);
      }
      const unsigned long long word = __ballot(o);
      if ((threadIdx.x & 63) == 0) d.obs[i4 >> 6] = word;
    }
  }
}
constexpr int kSubChunk = 8;  // subsamples per unrolled group in the data passes
__device__ __forceinline__ bool observed(const ChainDev& d, uint32_t i4) {
  return HMC_OBSMASK == 0 || ((d.obs[i4 >> 6] >> (i4 & 63)) & 1ull);
}

__global__ void __launch_bounds__(kWideThreads) k_coeff(const ChainDev* __restrict__ ch,
                                                         int nch, int total) {
  __shared__ double red[kWideThreads / 64];
  __shared__ float cb2n[kMaxSub], cb[kMaxSub], cn[kMaxSub];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    if (threadIdx.x < d.nsub) {
      const float bl = (float)d.P[kBias + threadIdx.x], nb = (float)d.P[kNbar + threadIdx.x];
      cb2n[threadIdx.x] = bl * bl * nb;
      cb[threadIdx.x] = bl;
      cn[threadIdx.x] = nb;
    }
    __syncthreads();
    const uint32_t nv4 = (uint32_t)(d.nv / 4), base4 = (uint32_t)lt * (kElemPerTile / 4);
    double acc = 0.0;
    for (uint32_t j = threadIdx.x; j < kElemPerTile / 4; j += kWideThreads) {
      const uint32_t i4 = base4 + j;
      if (i4 >= nv4) break;
      f4v al = {0.f, 0.f, 0.f, 0.f}, be = {0.f, 0.f, 0.f, 0.f};
      if (observed(d, i4)) {  // outside the support R^l = 0: alpha = beta = 0, no loads
        for (int l0 = 0; l0 < d.nsub; l0 += kSubChunk) {  // a chunk's loads in flight together
#pragma unroll
          for (int u = 0; u < kSubChunk; ++u) {
            const int l = l0 + u;
            if (l >= d.nsub) break;
            const f4v r = gld4(d.R + (size_t)l * d.nv, i4);
            const f4v c = gld4(d.counts + (size_t)l * d.nv, i4);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              if (r[q] > 0.f) {
                al[q] += cb2n[l] * r[q];
                be[q] += cb[l] * (c[q] - cn[l] * r[q]);
              }
            }
          }
        }
        if (d.growth) {  // per-voxel growth factor: b -> b D+ in the data model
          const f4v g = gld4(d.growth, i4);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            al[q] *= g[q] * g[q];
            be[q] *= g[q];
          }
        }
      }
      gst4(d.alpha, i4, al);
      gst4(d.beta, i4, be);
      acc += (double)al[0] + (double)al[1] + (double)al[2] + (double)al[3];
    }
    const double s = block_sum_w<kWideThreads / 64>(acc, red);
    if (threadIdx.x == 0) d.part[kPartAlpha * d.maxtiles + lt] = s;
    __syncthreads();
  }
}

// sum of alpha per tile (caller-installed coefficients)
__global__ void __launch_bounds__(kThreads) k_alpha_sum(const ChainDev* __restrict__ ch, int nch,
                                                         int total) {
  __shared__ double red[4];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    double acc = 0.0;
    for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
      const long long i = (long long)lt * kElemPerTile + j;
      if (i >= d.nv) break;
      acc += d.alpha[i];
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) d.part[kPartAlpha * d.maxtiles + lt] = s;
    __syncthreads();
  }
}

// S0 = sum R, B = sum N^2/R, N_obs per subsample (R > 0): mpart[tile][3 l + {0,1,2}]
__global__ void __launch_bounds__(kThreads) k_static_moments(const ChainDev* __restrict__ ch,
                                                              int nch, int total) {
  __shared__ double red[4];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    for (int l = 0; l < d.nsub; ++l) {
      double s0 = 0.0, sb = 0.0, so = 0.0;
      for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
        const long long i = (long long)lt * kElemPerTile + j;
        if (i >= d.nv) break;
        const float r = d.R[(size_t)l * d.nv + i];
        if (r > 0.f) {
          const double c = d.counts[(size_t)l * d.nv + i];
          s0 += r;
          sb += c * c / (double)r;
          so += 1.0;
        }
      }
      s0 = block_sum(s0, red);
      sb = block_sum(sb, red);
      so = block_sum(so, red);
      if (threadIdx.x == 0) {
        double* o = d.mpart + (size_t)lt * 3 * d.nsub + 3 * l;
        o[0] = s0;
        o[1] = sb;
        o[2] = so;
      }
    }
    __syncthreads();
  }
}

// S1 = sum R delta, S2 = sum R delta^2, T = sum N delta per subsample (R > 0).
// Subsamples go in chunks of kSubChunk per pass over the tile: a thread keeps the
// chunk's 3 kSubChunk sums in registers and has the chunk's loads in flight
// together; per sum the block reduction is block_sum's (butterfly per wave, waves
// added in order).
__global__ void __launch_bounds__(kThreads) k_moments(const ChainDev* __restrict__ ch, int nch,
                                                       int total) {
  constexpr int V = 3 * kSubChunk;
  __shared__ double red[4 * V];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    const uint32_t nv4 = (uint32_t)(d.nv / 4), base4 = (uint32_t)lt * (kElemPerTile / 4);
    for (int l0 = 0; l0 < d.nsub; l0 += kSubChunk) {
      double sm[V];
#pragma unroll
      for (int u = 0; u < V; ++u) sm[u] = 0.0;
      for (uint32_t j = threadIdx.x; j < kElemPerTile / 4; j += kThreads) {
        const uint32_t i4 = base4 + j;
        if (i4 >= nv4) break;
        if (!observed(d, i4)) continue;  // R^l = 0 on all 4 voxels: no contribution
        const f4v x = gld4(d.dr, i4);
        const f4v g = d.growth ? gld4(d.growth, i4) : f4v{1.f, 1.f, 1.f, 1.f};
#pragma unroll
        for (int u = 0; u < kSubChunk; ++u) {
          const int l = l0 + u;
          if (l >= d.nsub) break;
          const f4v r = gld4(d.R + (size_t)l * d.nv, i4);
          const f4v c = gld4(d.counts + (size_t)l * d.nv, i4);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (r[q] > 0.f) {
              const double xq = (double)x[q] * (double)g[q];  // D+ delta
              sm[3 * u] += (double)r[q] * xq;
              sm[3 * u + 1] += (double)r[q] * xq * xq;
              sm[3 * u + 2] += (double)c[q] * xq;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < V; ++u) sm[u] = wave_sum(sm[u]);
      __syncthreads();  // red of the previous chunk / tile consumed
      if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int u = 0; u < V; ++u) red[(threadIdx.x >> 6) * V + u] = sm[u];
      }
      __syncthreads();
      const int nl = d.nsub - l0 < kSubChunk ? d.nsub - l0 : kSubChunk;
      if ((int)threadIdx.x < 3 * nl) {
        const int u = threadIdx.x;
        d.mpart[(size_t)lt * 3 * d.nsub + 3 * l0 + u] =
            red[u] + red[V + u] + red[2 * V + u] + red[3 * V + u];
      }
    }
    __syncthreads();
  }
}

// data energy on delta_r
__global__ void __launch_bounds__(kThreads) k_energy_r(const ChainDev* __restrict__ ch, int nch,
                                                        int total) {
  __shared__ double red[4];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    double acc = 0.0;
    for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
      const long long i = (long long)lt * kElemPerTile + j;
      if (i >= d.nv) break;
      const double x = d.dr[i];
      acc += (0.5 * d.alpha[i] * x - d.beta[i]) * x;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) d.part[kPartDat * d.maxtiles + lt] = s;
    __syncthreads();
  }
}

__device__ __forceinline__ void kindex(long long i, int n, int* fx, int* fy, int* kz) {
  // i < N^2 (N/2 + 1) < 2^31 for every supported N: 32-bit unsigned arithmetic
  const uint32_t u = (uint32_t)i, h = (uint32_t)(n / 2 + 1), un = (uint32_t)n;
  const uint32_t r = u / h, x = r / un;
  *kz = (int)(u - r * h);
  *fy = sfreq((int)(r - x * un), n);
  *fx = sfreq((int)x, n);
}

// kinetic and prior energies on mom_k, delta_k
__global__ void __launch_bounds__(kThreads) k_energy_k(const ChainDev* __restrict__ ch, int nch,
                                                        int total) {
  __shared__ double red[4];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileK)];
    const int lt = tile - d.tb[kTileK];
    double ak = 0.0, ap = 0.0;
    for (int j = threadIdx.x; j < kElemPerTile; j += kThreads) {
      const long long i = (long long)lt * kElemPerTile + j;
      if (i >= d.nh) break;
      int fx, fy, kz;
      kindex(i, d.n, &fx, &fy, &kz);
      const int m = shell_of(d, fx, fy, kz);
      if (m < 0) continue;
      const double w = (kz == 0 || kz == d.n / 2) ? 1.0 : 2.0;
      const float2 p = d.pk[i], x = d.dk[i];
      ak += w * ((double)p.x * p.x + (double)p.y * p.y) * d.td[kDInvMass + m];
      ap += w * ((double)x.x * x.x + (double)x.y * x.y) * d.td[kDInvLam + m];
    }
    const double sk = block_sum(0.5 * ak, red);
    const double sp = block_sum(0.5 * ap, red);
    if (threadIdx.x == 0) {
      d.part[kPartKin * d.maxtiles + lt] = sk;
      d.part[kPartPri * d.maxtiles + lt] = sp;
    }
    __syncthreads();
  }
}

// shell sums sigma_m and mode counts n_m (full-grid weights) per tile
// Per-shell sums over k-space tiles into shpart[m][tile] (weights w = 1 on the
// kz = 0, N/2 planes, 2 elsewhere; k = 0 excluded) through per-wave LDS bins; the
// shell index comes from the branch-free integer rule (no table loads):
//   SP_POWER: sum w |delta_hat|^2 (sigma_m), with counts also sum w (mode counts,
//             into mpart; init only, the sweep's P draw needs sigma alone);
//   SP_DOT:   sum w Re(conj(delta_hat) g_hat) of the stored state and gradient
//             (the joint move's dU at its start).
enum ShellSum : int { SP_POWER = 0, SP_DOT = 1 };
constexpr int kShellWaves = kWideThreads / 64;

// One tile of kElemPerTile modes of a field dk (and gk for SP_DOT) into sig[m * sstride]
// and, when cnt_out is set, the mode counts into cnt_out[m]; bins and cnt are the
// block's LDS bins (one copy per wave), summed in a fixed order (reproducible).
template <int WHAT>
__device__ __forceinline__ void shell_sum_tile(const float2* __restrict__ dk,
                                               const float2* __restrict__ gk, int n, int nb,
                                               long long nh, int lt, double* sig, size_t sstride,
                                               double* cnt_out, double* bins, double* cnt) {
  const bool with_counts = cnt_out != nullptr;
  for (int i = threadIdx.x; i < kShellWaves * kMaxBins; i += kWideThreads) {
    bins[i] = 0.0;
    cnt[i] = 0.0;
  }
  __syncthreads();
  const int wv = (threadIdx.x >> 6) * kMaxBins;
  const uint32_t qmax = 3u * (uint32_t)(n / 2) * (uint32_t)(n / 2), nbu = (uint32_t)nb;
  const float inv_qmax = 1.f / (float)qmax;
  for (int j = threadIdx.x; j < kElemPerTile; j += kWideThreads) {
    const long long i = (long long)lt * kElemPerTile + j;
    if (i >= nh) break;
    int fx, fy, kz;
    kindex(i, n, &fx, &fy, &kz);
    const int m = shell_fast((uint32_t)(fx * fx + fy * fy + kz * kz), qmax, inv_qmax, nbu);
    if (m < 0) continue;
    const double w = (kz == 0 || kz == n / 2) ? 1.0 : 2.0;
    const float2 x = dk[i];
    double val;
    if constexpr (WHAT == SP_POWER) {
      val = w * ((double)x.x * x.x + (double)x.y * x.y);
    } else {
      const float2 g = gk[i];
      val = w * ((double)x.x * g.x + (double)x.y * g.y);
    }
    atomicAdd(&bins[wv + m], val);
    if (WHAT == SP_POWER && with_counts) atomicAdd(&cnt[wv + m], w);
  }
  __syncthreads();
  for (int m = threadIdx.x; m < nb; m += kWideThreads) {
    double sb = 0.0, sc = 0.0;
#pragma unroll
    for (int c = 0; c < kShellWaves; ++c) {  // fixed order: reproducible
      sb += bins[c * kMaxBins + m];
      sc += cnt[c * kMaxBins + m];
    }
    sig[(size_t)m * sstride] = sb;
    if (WHAT == SP_POWER && with_counts) cnt_out[m] = sc;
  }
  __syncthreads();
}

template <int WHAT>
__global__ void __launch_bounds__(kWideThreads) k_shell_sum(const ChainDev* __restrict__ ch,
                                                            int nch, int total, int with_counts) {
  // one bin copy per wave; 1024-thread blocks keep 16 waves per tile in flight
  // (the per-mode work is a dependent chain of index arithmetic, not bandwidth)
  __shared__ double bins[kShellWaves * kMaxBins];
  __shared__ double cnt[kShellWaves * kMaxBins];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileK)];
    const int lt = tile - d.tb[kTileK];
    shell_sum_tile<WHAT>(d.dk, d.gk, d.n, d.nb, d.nh, lt, d.shpart + lt, d.maxtiles,
                         (WHAT == SP_POWER && with_counts) ? d.mpart + (size_t)lt * d.nb : nullptr,
                         bins, cnt);
  }
}

__global__ void __launch_bounds__(kThreads) k_shell_index(const ChainDev* __restrict__ ch,
                                                           int total, int16_t* out) {
  const ChainDev& d = ch[0];
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < d.nh;
       i += (long long)gridDim.x * kThreads) {
    int fx, fy, kz;
    kindex(i, d.n, &fx, &fy, &kz);
    out[i] = (int16_t)shell_of(d, fx, fy, kz);
  }
}

// Accept/reject bookkeeping on the device: after a density trajectory,
// rejected chains restore delta_hat and g_hat from the backups, accepted chains
// take the proposal's real field.  After a joint move, accepted chains rescale
// delta_hat per shell and take the move's g_hat and real field.
// k-space arrays move two complex entries (16 bytes) per access: N^2 (N/2 + 1)
// and the tile size are even
__global__ void __launch_bounds__(kWideThreads) k_commit_k(const ChainDev* __restrict__ ch,
                                                            int nch, int total, int what) {
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileK)];
    const int lt = tile - d.tb[kTileK];
    const bool acc = what == C_HMC ? d.P[kAcc] != 0.0 : d.P[kRjAcc] != 0.0;
    if (what == C_HMC && acc) continue;
    if (what == C_RJ && !acc) continue;
    const uint32_t nh2 = (uint32_t)(d.nh / 2), base2 = (uint32_t)lt * (kElemPerTile / 2);
    float* dk = (float*)d.dk;
    float* gk = (float*)d.gk;
    for (uint32_t j = threadIdx.x; j < kElemPerTile / 2; j += kWideThreads) {
      const uint32_t i2 = base2 + j;
      if (i2 >= nh2) break;
      gst4(gk, i2, gld4((const float*)d.bgk, i2));
      if (what == C_HMC) {
        gst4(dk, i2, gld4((const float*)d.bdk, i2));
      } else {
        f4v v = gld4(dk, i2);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          int fx, fy, kz;
          kindex(2 * (long long)i2 + e, d.n, &fx, &fy, &kz);
          const int m = shell_of(d, fx, fy, kz);
          const float sc = m >= 0 ? d.tf[kTScale + m] : 0.f;
          v[2 * e] *= sc;
          v[2 * e + 1] *= sc;
        }
        gst4(dk, i2, v);
      }
    }
  }
}
__global__ void __launch_bounds__(kWideThreads) k_commit_r(const ChainDev* __restrict__ ch,
                                                            int nch, int total, int what) {
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const ChainDev& d = ch[find_chain(ch, nch, tile, kTileR)];
    const int lt = tile - d.tb[kTileR];
    const bool acc = what == C_HMC ? d.P[kAcc] != 0.0 : d.P[kRjAcc] != 0.0;
    if (!acc) continue;
    const uint32_t nv4 = (uint32_t)(d.nv / 4), base4 = (uint32_t)lt * (kElemPerTile / 4);
    for (uint32_t j = threadIdx.x; j < kElemPerTile / 4; j += kWideThreads) {
      const uint32_t i4 = base4 + j;
      if (i4 >= nv4) break;
      gst4(d.dr, i4, gld4(d.drn, i4));
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_copy_real(const ChainDev* __restrict__ ch,
                                                         int total, const float* src, float* dst) {
  const ChainDev& d = ch[0];
  for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < d.nv;
       i += (long long)gridDim.x * kThreads)
    dst[i] = src[i];
}

// ------------------------------------------------------------------ per-chain scalar kernels
__device__ double tile_sum(const double* p, int n, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) acc += p[i];
  return block_sum(acc, red);
}

__global__ void __launch_bounds__(kThreads) k_reduce_slot(const ChainDev* __restrict__ ch,
                                                           int slot, int dst, int cls, int mean) {
  __shared__ double red[4];
  const ChainDev& d = ch[blockIdx.x];
  const double s = tile_sum(d.part + (size_t)slot * d.maxtiles, d.nt[cls], red);
  if (threadIdx.x == 0) d.P[dst] = mean ? s / (double)d.nv : s;
}

// Column sums of per-tile partials (src 0: shpart [shell][tile]; src 1: mpart
// [tile][width]), one block per (column, chain), fixed order (strided per thread,
// then the block tree).
__device__ __forceinline__ double column_sum(const double* p, size_t step, int nt, double* red) {
  double acc = 0.0;
  for (int t = threadIdx.x; t < nt; t += kThreads) acc += p[(size_t)t * step];
  return block_sum(acc, red);
}
// mode 0: P[dst + q] = sum (per-shell tables, width nb)
// mode 1: P[dst + (q % 3) * kMaxSub + q / 3] = sum (moments, width 3 nsub)
// mode 2: P[dst + q] = sum / 2 + (alpha_prior - 1) (joint-move dU, width nb)
__global__ void __launch_bounds__(kThreads) k_colsum(const ChainDev* __restrict__ ch, int src,
                                                      int cls, int dst, int mode) {
  __shared__ double red[4];
  const ChainDev& d = ch[blockIdx.y];
  const int q = blockIdx.x;
  const int width = mode == 1 ? 3 * d.nsub : d.nb;
  if (q >= width) return;
  // shell partials are [shell][tile] (a block reads one contiguous row), the
  // others [tile][width]
  const double s = src == 0 ? column_sum(d.shpart + (size_t)q * d.maxtiles, 1, d.nt[cls], red)
                            : column_sum(d.mpart + q, (size_t)width, d.nt[cls], red);
  if (threadIdx.x == 0) {
    if (mode == 0) d.P[dst + q] = s;
    else if (mode == 1) d.P[dst + (q % 3) * kMaxSub + q / 3] = s;
    else d.P[dst + q] = 0.5 * s + (d.alpha_prior - 1.0);
  }
}

// shell tables from lambda and mean(alpha): 1/lambda, 1/m, sqrt(m), m = 1/lambda + abar
__global__ void k_tables(const ChainDev* __restrict__ ch) {
  const ChainDev& d = ch[blockIdx.x];
  const double abar = d.P[kAbar];
  for (int m = threadIdx.x; m < d.nb; m += blockDim.x) {
    const double il = 1.0 / d.P[kLam + m];
    // plain mass m_k = 1/lambda + mean(alpha); the real-space diagonal variant
    // M^-1 = P diag(v) P takes m_k = 1/mean(v) for every mode (with D = v/mean(v))
    const double ms = d.mass_flat ? 1.0 / d.P[kLmean] : il + abar;
    d.td[kDInvLam + m] = il;
    d.td[kDInvMass + m] = 1.0 / ms;
    d.tf[kTInvLam + m] = (float)il;
    d.tf[kTInvMass + m] = (float)(1.0 / ms);
    d.tf[kTSqrtMass + m] = (float)sqrt(ms);
    d.tf[kTScale + m] = 1.f;
  }
}

// Metropolis test of eq. acceptance_rule: accept iff ln u < -dH (u: Philox stream 4)
__global__ void k_accept(const ChainDev* __restrict__ ch) {
  const ChainDev& d = ch[blockIdx.x];
  if (threadIdx.x != 0) return;
  const uint32_t traj = *d.draw;
  const double H0 = d.P[kK0] + d.P[kPi0] + d.P[kDcur];
  const double H1 = d.P[kK1] + d.P[kPi1] + d.P[kD1];
  const double dH = H1 - H0;
  const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, hmcrng::kAccept, traj, 0, 0);
  const double lu = log(hmcrng::uniform(w.w[0]));
  const bool finite = isfinite(dH);
  const bool acc = finite && lu < -dH;
  d.P[kDH] = dH;
  d.P[kLogU] = lu;
  d.P[kAcc] = acc ? 1.0 : 0.0;
  d.P[kStatus] = finite ? 0.0 : 1.0;
  if (acc) d.P[kDcur] = d.P[kD1];
}

// P_m | delta: lambda_m = sigma_m / x_m, x_m ~ chi^2(n_m + 2 alpha - 2) = 2 Gamma(.)
__global__ void k_draw_power(const ChainDev* __restrict__ ch) {
  const ChainDev& d = ch[blockIdx.x];
  const uint32_t sweep = *d.draw;
  for (int m = threadIdx.x; m < d.nb; m += blockDim.x) {
    const double nm = d.P[kNmodes + m];
    // an empty shell or a field with no power in it leaves P_m unchanged
    if (nm <= 0.0 || !(d.P[kSigma + m] > 0.0)) continue;
    const double beta = nm + 2.0 * d.alpha_prior - 2.0;
    const double g = hmcsamp::gamma_mt(0.5 * beta, d.seed, d.chain, sweep, (uint32_t)m);
    if (g > 0.0)
      d.P[kLam + m] = d.P[kSigma + m] / (2.0 * g);
    else
      d.P[kStatus] = 2.0;
  }
}

// Nbar^l ~ GIG(1 - N_obs/2, A, B), then b^l ~ N(D/C, 1/C) with the new Nbar^l
__global__ void k_draw_nbar_bias(const ChainDev* __restrict__ ch) {
  const ChainDev& d = ch[blockIdx.x];
  const uint32_t sweep = *d.draw;
  for (int l = threadIdx.x; l < d.nsub; l += blockDim.x) {
    const double b = d.P[kBias + l];
    const double S0 = d.P[kS0 + l], Bs = d.P[kBsum + l], nobs = d.P[kNobs + l];
    const double S1 = d.P[kS1 + l], S2 = d.P[kS2 + l], Ts = d.P[kTsum + l];
    const double A = S0 + 2.0 * b * S1 + b * b * S2;
    const double nb = hmcsamp::gig(1.0 - 0.5 * nobs, A, Bs, d.seed, d.chain, sweep, (uint32_t)l);
    if (nb > 0.0)
      d.P[kNbar + l] = nb;
    else
      d.P[kStatus] = 3.0;
    if (!((d.fixed_mask >> l) & 1u) && S2 > 0.0) {  // S2 = 0: degenerate, b kept
      const double nbl = d.P[kNbar + l];
      const double C = nbl * S2, D = Ts - nbl * S1;
      const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, hmcrng::kBias, sweep, (uint32_t)l, 0);
      double z, unused;
      hmcrng::box_muller(w.w[0], w.w[1], &z, &unused);
      d.P[kBias + l] = D / C + z / sqrt(C);
    }
  }
}

// Joint (P, delta) move: HMC in theta_m = ln lambda_m at fixed whitened field.
// The mass max(1, n_m lambda_ref,m mean(alpha) / 4) takes lambda_ref at the centre
// of the walls (the lambda the chain started from), never the current theta: the
// move must run the same leapfrog map from either end for detailed balance.
// BEGIN: theta0, mass, momenta (stream 8), H0, first half kick and drift.
// STEP:  kick with dU at the current theta, drift.
// END:   last half kick, H1, Metropolis test (stream 9), lambda update.
// dU_m = 1/2 sum_{k in m} w Re(conj(delta_hat) g_hat) + (alpha - 1) from the tile partials.
// Mirror th into [lo, hi], negating rho once per reflection; returns the count.
__device__ int rj_reflect(double* th, double* rho, double lo, double hi) {
  int hits = 0;
  for (int it = 0; it < 64; ++it) {
    if (*th > hi) {
      *th = 2.0 * hi - *th;
    } else if (*th < lo) {
      *th = 2.0 * lo - *th;
    } else {
      break;
    }
    *rho = -*rho;
    ++hits;
  }
  return hits;
}

__global__ void __launch_bounds__(kThreads) k_rj(const ChainDev* __restrict__ ch, int phase) {
  __shared__ double red[4];
  const ChainDev& d = ch[blockIdx.x];
  const uint32_t sweep = *d.draw;
  const double am1 = d.alpha_prior - 1.0;
  const int m = threadIdx.x;
  const bool on = m < d.nb;
  const double dU = on ? d.P[kDU + m] : 0.0;
  const double eps = d.eps;
  if (phase == RJ_BEGIN) {
    double th = 0.0, rho = 0.0, ms = 1.0;
    if (on) {
      th = log(d.P[kLam + m]);
      const double lam_ref = exp(0.5 * (d.P[kLo + m] + d.P[kHi + m]));
      ms = fmax(1.0, 0.25 * d.P[kNmodes + m] * lam_ref * d.P[kAbar]);
      const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, hmcrng::kRjMomenta, sweep, 0,
                                         (uint32_t)(m >> 2));
      double z0, z1;
      if ((m & 2) == 0)
        hmcrng::box_muller(w.w[0], w.w[1], &z0, &z1);
      else
        hmcrng::box_muller(w.w[2], w.w[3], &z0, &z1);
      rho = sqrt(ms) * ((m & 1) ? z1 : z0);
      d.P[kTheta0 + m] = th;
      d.P[kMth + m] = ms;
    }
    const double k0 = block_sum(on ? 0.5 * rho * rho / ms : 0.0, red);
    const double st = block_sum(on ? th : 0.0, red);
    if (m == 0) {
      d.P[kRjK0] = k0;
      d.P[kRjU0] = d.P[kDcur] + am1 * st;
    }
    if (on) {
      rho -= 0.5 * eps * dU;
      th += eps * rho / ms;
      d.P[kWall + m] = (double)rj_reflect(&th, &rho, d.P[kLo + m], d.P[kHi + m]);
      d.P[kTheta + m] = th;
      d.P[kRho + m] = rho;
      d.tf[kTScale + m] = (float)exp(0.5 * (th - d.P[kTheta0 + m]));
    }
  } else if (phase == RJ_STEP) {
    if (on) {
      double th = d.P[kTheta + m], rho = d.P[kRho + m];
      const double ms = d.P[kMth + m];
      rho -= eps * dU;
      th += eps * rho / ms;
      d.P[kWall + m] += (double)rj_reflect(&th, &rho, d.P[kLo + m], d.P[kHi + m]);
      d.P[kTheta + m] = th;
      d.P[kRho + m] = rho;
      d.tf[kTScale + m] = (float)exp(0.5 * (th - d.P[kTheta0 + m]));
    }
  } else {
    double th = 0.0, rho = 0.0, ms = 1.0;
    if (on) {
      th = d.P[kTheta + m];
      ms = d.P[kMth + m];
      rho = d.P[kRho + m] - 0.5 * eps * dU;
    }
    const double k1 = block_sum(on ? 0.5 * rho * rho / ms : 0.0, red);
    const double st = block_sum(on ? th : 0.0, red);
    const double hits = block_sum(on ? d.P[kWall + m] : 0.0, red);
    __shared__ int acc_s;
    if (m == 0) {
      d.P[kRjHits] = hits;
      const double H0 = d.P[kRjK0] + d.P[kRjU0];
      const double H1 = k1 + d.P[kD1] + am1 * st;
      const double dH = H1 - H0;
      const hmcrng::U4 w = hmcrng::block(d.seed, d.chain, hmcrng::kRjAccept, sweep, 0, 0);
      const double lu = log(hmcrng::uniform(w.w[0]));
      const bool acc = isfinite(dH) && lu < -dH;
      d.P[kRjDH] = dH;
      d.P[kRjAcc] = acc ? 1.0 : 0.0;
      if (acc) d.P[kDcur] = d.P[kD1];
      acc_s = acc;
    }
    __syncthreads();
    if (on && acc_s) d.P[kLam + m] = exp(th);
  }
}

// ------------------------------------------------------------------ launch wrappers
static inline int eg(int total) { return total < 4096 ? total : 4096; }

template <int N>
static void launch_xl_n(int mode, dim3 g, dim3 bl, int lds, hipStream_t s, const ChainDev* ch,
                        int nch, int total, XArgs a, const float2* tw) {
  switch (mode) {
    case L_START: hipLaunchKernelGGL((k_xpass_l_n<N, L_START>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_DRIFT: hipLaunchKernelGGL((k_xpass_l_n<N, L_DRIFT>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_KICK: hipLaunchKernelGGL((k_xpass_l_n<N, L_KICK>), g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_KICK_LAST:
      hipLaunchKernelGGL((k_xpass_l_n<N, L_KICK_LAST>), g, bl, lds, s, ch, nch, total, a, tw);
      break;
  }
}
void launch_xpass_learned(int mode, const ChainDev* ch, int nch, int total, int lds, XArgs a,
                          const float2* tw, int cap, hipStream_t s, int uniform_n) {
  dim3 g(grid_of(total, cap)), bl(kThreads);
  switch (uniform_n) {
#define C(NN) case NN: launch_xl_n<NN>(mode, g, bl, lds, s, ch, nch, total, a, tw); return;
    HMC_FOR_N(C)
#undef C
    default: break;
  }
  switch (mode) {
    case L_START: hipLaunchKernelGGL(k_xpass_l<L_START>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_DRIFT: hipLaunchKernelGGL(k_xpass_l<L_DRIFT>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_KICK: hipLaunchKernelGGL(k_xpass_l<L_KICK>, g, bl, lds, s, ch, nch, total, a, tw); break;
    case L_KICK_LAST:
      hipLaunchKernelGGL(k_xpass_l<L_KICK_LAST>, g, bl, lds, s, ch, nch, total, a, tw);
      break;
  }
}
void launch_zpass_learned(int mode, const ChainDev* ch, int nch, int total, int lds, ZArgs a,
                          const float2* tw, int cap, hipStream_t s, int uniform_n) {
  dim3 g(grid_of(total, cap)), bl(kThreads);
  switch (uniform_n) {
#define C(NN)                                                                               \
  case NN:                                                                                  \
    if (mode == LZ_FORCE)                                                                   \
      hipLaunchKernelGGL((k_zpass_l_n<NN, LZ_FORCE>), g, bl, lds, s, ch, nch, total, a, tw); \
    else                                                                                    \
      hipLaunchKernelGGL((k_zpass_l_n<NN, LZ_VEL>), g, bl, lds, s, ch, nch, total, a, tw);   \
    return;
    HMC_FOR_N(C)
#undef C
    default: break;
  }
  if (mode == LZ_FORCE)
    hipLaunchKernelGGL(k_zpass_l<LZ_FORCE>, g, bl, lds, s, ch, nch, total, a, tw);
  else
    hipLaunchKernelGGL(k_zpass_l<LZ_VEL>, g, bl, lds, s, ch, nch, total, a, tw);
}
void launch_mass_prep(int phase, const ChainDev* ch, int total_r, const float* logvar,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_mass_prep, dim3(eg(total_r)), dim3(kThreads), 0, s, ch, total_r, logvar,
                     phase);
}
void launch_shell_lut(const ChainDev* ch, int n, hipStream_t s) {
  const int q = 3 * (n / 2) * (n / 2) + 1;
  hipLaunchKernelGGL(k_shell_lut, dim3((q + kThreads - 1) / kThreads), dim3(kThreads), 0, s, ch);
}
void launch_export(const ChainDev* ch, int nch, int sweep, double* rec, int32_t* acc,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3(nch), dim3(128), 0, s, ch, nch, sweep, rec, acc);
}
// Running per-voxel mean and sum of squared deviations of a float field over
// `count` samples (Welford's update, float64 accumulators); count = 1 starts them.
__global__ void __launch_bounds__(kThreads) k_field_moments(const float* __restrict__ x,
                                                            double* __restrict__ mean,
                                                            double* __restrict__ m2, long long nv,
                                                            long long count) {
  const double inv = 1.0 / (double)count;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
    const double v = (double)x[i];
    if (count == 1) {
      mean[i] = v;
      m2[i] = 0.0;
    } else {
      const double d = v - mean[i];
      const double mn = mean[i] + d * inv;
      mean[i] = mn;
      m2[i] += d * (v - mn);
    }
  }
}
void launch_field_moments(const float* x, double* mean, double* m2, long long nv, long long count,
                          hipStream_t s) {
  const long long blocks = (nv + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_field_moments, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(kThreads),
                     0, s, x, mean, m2, nv, count);
}
void launch_warm_combine(const ChainDev* ch, int total_r, const float* mu, const float* logvar,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_warm_combine, dim3(eg(total_r)), dim3(kThreads), 0, s, ch, total_r, mu,
                     logvar);
}
void launch_coeff(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_coeff, dim3(eg(total)), dim3(kWideThreads), 0, s, ch, nch, total);
}
void launch_alpha_sum(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_alpha_sum, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_static_moments(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_static_moments, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_obs_mask(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_obs_mask, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_moments(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_moments, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_energy_k(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_k, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_energy_r(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_r, dim3(eg(total)), dim3(kThreads), 0, s, ch, nch, total);
}
void launch_shell_power(const ChainDev* ch, int nch, int total, hipStream_t s, int with_counts) {
  hipLaunchKernelGGL(k_shell_sum<SP_POWER>, dim3(eg(total)), dim3(kWideThreads), 0, s, ch, nch,
                     total, with_counts);
}
void launch_shell_dot(const ChainDev* ch, int nch, int total, hipStream_t s) {
  hipLaunchKernelGGL(k_shell_sum<SP_DOT>, dim3(eg(total)), dim3(kWideThreads), 0, s, ch, nch, total,
                     0);
}
void launch_shell_index(const ChainDev* ch, int total, int16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_shell_index, dim3(eg(total)), dim3(kThreads), 0, s, ch, total, out);
}
void launch_commit(int what, const ChainDev* ch, int nch, int total_k, int total_r,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_commit_k, dim3(eg(total_k)), dim3(kWideThreads), 0, s, ch, nch, total_k,
                     what);
  hipLaunchKernelGGL(k_commit_r, dim3(eg(total_r)), dim3(kWideThreads), 0, s, ch, nch, total_r,
                     what);
}
void launch_copy_real(const ChainDev* ch, int total_r, const float* src, float* dst,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_copy_real, dim3(eg(total_r)), dim3(kThreads), 0, s, ch, total_r, src,
                     dst);
}
void launch_reduce_slot(const ChainDev* ch, int nch, int slot, int dst, int cls, hipStream_t s,
                        bool mean) {
  hipLaunchKernelGGL(k_reduce_slot, dim3(nch), dim3(kThreads), 0, s, ch, slot, dst, cls,
                     mean ? 1 : 0);
}
void launch_colsum(const ChainDev* ch, int nch, int width, int src, int cls, int dst, int mode,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(width, nch), dim3(kThreads), 0, s, ch, src, cls, dst, mode);
}
void launch_tables(const ChainDev* ch, int nch, hipStream_t s) {
  hipLaunchKernelGGL(k_tables, dim3(nch), dim3(kMaxBins), 0, s, ch);
}
__global__ void k_set_draw(uint32_t* p, uint32_t v) {
  if (threadIdx.x == 0) *p = v;
}
void launch_set_draw(uint32_t* p, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_draw, dim3(1), dim3(64), 0, s, p, v);
}
void launch_accept(const ChainDev* ch, int nch, hipStream_t s) {
  hipLaunchKernelGGL(k_accept, dim3(nch), dim3(64), 0, s, ch);
}
void launch_draw_power(const ChainDev* ch, int nch, hipStream_t s) {
  hipLaunchKernelGGL(k_draw_power, dim3(nch), dim3(kMaxBins), 0, s, ch);
}
void launch_draw_nbar_bias(const ChainDev* ch, int nch, hipStream_t s) {
  hipLaunchKernelGGL(k_draw_nbar_bias, dim3(nch), dim3(64), 0, s, ch);
}
void launch_rj(int phase, const ChainDev* ch, int nch, int nb_max, hipStream_t s, int cls) {
  launch_colsum(ch, nch, nb_max, 0, cls, kDU, 2, s);  // dU from the per-tile shell dots
  hipLaunchKernelGGL(k_rj, dim3(nch), dim3(kThreads), 0, s, ch, phase);
}

}  // namespace hmc

// ------------------------------------------------------------------ no-allocation shell sums
// shell_power_noalloc: the shell sums of a caller's half-complex field without a
// context.  Its per-tile partial sums live in `scratch`, a file-scope device array
// (one copy per GPU, held until the process ends); host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
namespace hmc {
namespace {
constexpr int kNoAllocMaxN = 256;
constexpr long long kNoAllocMaxModes = (long long)kNoAllocMaxN * kNoAllocMaxN * (kNoAllocMaxN / 2 + 1);
constexpr int kNoAllocMaxTiles = (int)((kNoAllocMaxModes + kElemPerTile - 1) / kElemPerTile);
// [shell][tile] sums of w |delta_hat|^2, then [tile][shell] mode counts
constexpr size_t kScratchDoubles = 2 * (size_t)kMaxBins * kNoAllocMaxTiles;
}  // namespace
}  // namespace hmc

static __device__ __align__(256) double scratch[hmc::kScratchDoubles];

namespace hmc {
namespace {

__global__ void __launch_bounds__(kWideThreads) k_shell_power_field(const float2* __restrict__ dk,
                                                                    int n, int nb, long long nh,
                                                                    int ntiles, double* part) {
  __shared__ double bins[kShellWaves * kMaxBins];
  __shared__ double cnt[kShellWaves * kMaxBins];
  double* cpart = part + (size_t)kMaxBins * ntiles;
  for (int lt = blockIdx.x; lt < ntiles; lt += gridDim.x)
    shell_sum_tile<SP_POWER>(dk, nullptr, n, nb, nh, lt, part + lt, (size_t)ntiles,
                             cpart + (size_t)lt * nb, bins, cnt);
}

// block (q, 0): sigma_q from the [shell][tile] row; block (q, 1): n_q from the
// [tile][shell] column; the same fixed order as the context's column sums
__global__ void __launch_bounds__(kThreads) k_shell_power_cols(const double* __restrict__ part,
                                                               int nb, int ntiles,
                                                               double* __restrict__ sigma,
                                                               int64_t* __restrict__ n_modes) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  if (blockIdx.y == 0) {
    const double s = column_sum(part + (size_t)q * ntiles, 1, ntiles, red);
    if (threadIdx.x == 0) sigma[q] = s;
  } else {
    const double s = column_sum(part + (size_t)kMaxBins * ntiles + q, (size_t)nb, ntiles, red);
    if (threadIdx.x == 0) n_modes[q] = (int64_t)s;
  }
}

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};  // device address of `scratch` per device id

}  // namespace
}  // namespace hmc

extern "C" hmc_status shell_power_noalloc(int32_t n, int32_t n_bins, const float* delta_k,
                                          double* sigma, int64_t* n_modes, void* stream) {
  using namespace hmc;
  if (!delta_k || !sigma) return record_free_error(HMC_EINVAL, "shell_power_noalloc: null pointer");
  if (!(n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 192 || n == 256))
    return record_free_error(HMC_EINVAL, "shell_power_noalloc: N must be 8, 16, 32, 64, 128, 192 or 256");
  if (n_bins < 1 || n_bins > kMaxBins)
    return record_free_error(HMC_EINVAL, "shell_power_noalloc: n_bins must be in 1..128");
  const long long nh = (long long)n * n * (n / 2 + 1);
  const int ntiles = (int)((nh + kElemPerTile - 1) / kElemPerTile);
  if (ntiles > kNoAllocMaxTiles)  // cannot happen for N <= 256; kept with the size checks
    return record_free_error(HMC_EINVAL, "shell_power_noalloc: grid exceeds the scratch array");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return record_free_error(HMC_EDEVICE, "shell_power_noalloc: no current device");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      const hipError_t e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_scratch_ptr[dev] = nullptr;
        return record_free_error(HMC_EDEVICE, "shell_power_noalloc: hipGetSymbolAddress failed");
      }
    }
    ptr = g_scratch_ptr[dev];
  }
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)ptr;
  hipLaunchKernelGGL(k_shell_power_field, dim3(eg(ntiles)), dim3(kWideThreads), 0, s,
                     (const float2*)delta_k, n, n_bins, nh, ntiles, part);
  hipLaunchKernelGGL(k_shell_power_cols, dim3(n_bins, n_modes ? 2 : 1), dim3(kThreads), 0, s, part,
                     n_bins, ntiles, sigma, n_modes);
  if (hipGetLastError() != hipSuccess)
    return record_free_error(HMC_EDEVICE, "shell_power_noalloc: launch failed");
  return HMC_OK;
}

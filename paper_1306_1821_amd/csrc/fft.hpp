// Device FFT building blocks for gfx950 (wave64).
//
// A pencil of length N is spread over T threads in a cyclic distribution:
// thread t holds elements t + T*e, e = 0..E-1 (E = N/T) in registers.  A
// Stockham autosort transform (radix list R_1..R_s, product N) keeps this
// property at both ends: the first stage reads the thread's own registers and
// the last stage writes its results back into the same registers, so global
// loads and stores are strided by T and coalesce across neighbouring pencils.
// Stages in between exchange through LDS (one write, barrier, one read).
//
// Stage with radix R after stages of total size Ns: butterfly j in [0, N/R)
// takes x[j + r N/R] (r < R), multiplies term r by W_{Ns R}^(r (j mod Ns)),
// applies a length-R DFT and writes y[(j - j mod Ns) R + j mod Ns + r Ns].
// Thread t runs butterflies j = t + T q, q < E/R, whose inputs are its
// registers q + r E/R.
//
// Twiddles W_N^i = exp(-2 pi i i/N) come from a float table built in float64
// on the host; small-radix constants are folded at compile time.
#pragma once
#include <hip/hip_runtime.h>

#ifndef HMC_TW_POW2
#define HMC_TW_POW2 1
#endif

namespace hmcfft {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex product with the fused multiply-adds written out: left to contraction,
// which of the two products gets fused depends on how the operands reach the
// expression (a load in the same block or a register from outside), so the same
// source could round differently in two kernels.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// -------------------------------------------------------------- compile-time trig
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double cx_sin_red(double x) {  // |x| <= pi
  double term = x, sum = x;
  for (int i = 1; i < 40; ++i) {
    term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    sum += term;
  }
  return sum;
}
// exp(-2 pi i e / R) for integer e (DIR = +1) or its conjugate (DIR = -1).
constexpr double cx_twc(int e, int R) {
  int m = ((e % R) + R) % R;
  double a = 2.0 * kPi * m / R;            // in [0, 2 pi)
  double b = a + 0.5 * kPi;                // cos(a) = sin(a + pi/2)
  if (b > kPi) b -= 2.0 * kPi;
  return cx_sin_red(b);
}
constexpr double cx_tws(int e, int R) {
  int m = ((e % R) + R) % R;
  double a = 2.0 * kPi * m / R;
  if (a > kPi) a -= 2.0 * kPi;
  return cx_sin_red(a);
}

// multiply by W_R^e (forward) or its conjugate (inverse), folded at compile time
template <int R, int E, int DIR>
__device__ __forceinline__ float2 ctw(float2 v) {
  constexpr int m = ((E % R) + R) % R;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (4 * m == R) {  // -i (fwd) / +i (inv)
    return DIR > 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  } else if constexpr (2 * m == R) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * m == 3 * R) {  // +i (fwd) / -i (inv)
    return DIR > 0 ? make_float2(-v.y, v.x) : make_float2(v.y, -v.x);
  } else {
    constexpr float c = (float)cx_twc(m, R);
    constexpr float s = (float)(-cx_tws(m, R));  // exp(-i a) = cos a - i sin a
    constexpr float sd = DIR > 0 ? s : -s;
    return make_float2(__builtin_fmaf(v.x, c, -(v.y * sd)), __builtin_fmaf(v.x, sd, v.y * c));
  }
}

// -------------------------------------------------------------- register DFTs
template <int R, int DIR>
struct DFT;

template <int DIR>
struct DFT<1, DIR> {
  __device__ __forceinline__ static void run(float2*) {}
};
template <int DIR>
struct DFT<2, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <int DIR>
struct DFT<3, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    // X1 = a0 + w a1 + w^2 a2, w = exp(-2 pi i/3): cos = -1/2, sin = -+sqrt(3)/2
    constexpr float h = 0.866025403784438646763723170752936183f;
    float2 s = cadd(v[1], v[2]);
    float2 d = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    // -i sqrt(3)/2 d (forward), +i sqrt(3)/2 d (inverse)
    float2 r = DIR > 0 ? make_float2(h * d.y, -h * d.x) : make_float2(-h * d.y, h * d.x);
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};
template <int DIR>
struct DFT<4, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    float2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    float2 r = ctw<4, 1, DIR>(d13);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, r);
    v[3] = csub(d02, r);
  }
};

// Composite length R1*R2 in registers: inner DFTs of length R1 on stride-R2
// subsequences, twiddle W_R^(n2 k1), outer DFTs of length R2.
template <int R1, int R2, int DIR>
struct DFTct {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr int R = R1 * R2;
    float2 tmp[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      float2 a[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[n1 * R2 + n2];
      DFT<R1, DIR>::run(a);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) tmp[k1 * R2 + n2] = a[k1];
    }
    apply_tw<0>(tmp);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 b[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) b[n2] = tmp[k1 * R2 + n2];
      DFT<R2, DIR>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = b[k2];
    }
  }
  template <int I>
  __device__ __forceinline__ static void apply_tw(float2* tmp) {
    if constexpr (I < R1 * R2) {
      constexpr int k1 = I / R2, n2 = I % R2;
      tmp[I] = ctw<R1 * R2, k1 * n2, DIR>(tmp[I]);
      apply_tw<I + 1>(tmp);
    }
  }
};

template <int DIR> struct DFT<6, DIR> : DFTct<2, 3, DIR> {};
template <int DIR> struct DFT<8, DIR> : DFTct<4, 2, DIR> {};
template <int DIR> struct DFT<12, DIR> : DFTct<4, 3, DIR> {};
template <int DIR> struct DFT<16, DIR> : DFTct<4, 4, DIR> {};

// -------------------------------------------------------------- radix lists
template <int... Rs>
struct Radices {};

// Plan for a length-N pencil on T threads.
template <int N_, int T_, typename RL>
struct Plan;
template <int N_, int T_, int... Rs>
struct Plan<N_, T_, Radices<Rs...>> {
  static constexpr int N = N_;
  static constexpr int T = T_;
  static constexpr int E = N_ / T_;
};

// One Stockham stage.  LDS element idx of this pencil is at lds[idx * es].
// LDS exchange ordering: a block barrier, or (WAVE) only a wavefront-scope fence
// when every pencil lives inside one wavefront (its LDS region is then touched by
// that wavefront alone, whose lanes run in lockstep)
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// PAD > 0 inserts one unused slot after every 2^PAD elements of the pencil
// (element i at lds[i * es + (i >> PAD)]): it spreads the stride-R writes of a
// stage over the LDS banks when a pencil is contiguous (es = 1).
template <int PAD>
__device__ __forceinline__ int lds_at(int i, int es) {
  if constexpr (PAD > 0) {
    return i * es + (i >> PAD);
  } else {
    return i * es;
  }
}

template <int N, int T, int R, int NS, int DIR, bool LAST, bool WAVE = false, int PAD = 0,
          bool DTW = false>
__device__ __forceinline__ void stage(float2* v, float2* lds, int es, int t, bool active,
                                      const float2* __restrict__ tw) {
  constexpr int E = N / T;
  constexpr int Q = E / R;
  static_assert(E % R == 0, "radix must divide the per-thread element count");
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = t + T * q;
    const int k = (NS == 1) ? 0 : (j % NS);
    float2 a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[q + r * Q];
    if constexpr (NS > 1) {
      constexpr int step = N / (NS * R);
#if HMC_TW_POW2
    if constexpr (N >= 128 && !DTW) {
      // large N: twiddles W^(r k) for every r from the table entries at powers of
      // two of r (at most three complex products each, fewer live registers)
      float2 wp[5];
#pragma unroll
      for (int b = 0; (1 << b) < R; ++b) wp[b] = tw[(1 << b) * k * step];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = make_float2(1.f, 0.f);
        bool first = true;
#pragma unroll
        for (int b = 0; (1 << b) < R; ++b)
          if (r & (1 << b)) {
            w = first ? wp[b] : cmul(w, wp[b]);
            first = false;
          }
        if (DIR < 0) w.y = -w.y;
        a[r] = cmul(a[r], w);
      }
    } else
#endif
    {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * step];
        if (DIR < 0) w.y = -w.y;
        a[r] = cmul(a[r], w);
      }
    }
    }
    DFT<R, DIR>::run(a);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * Q] = a[r];
    } else {
      if (active) {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_at<PAD>((j - k) * R + k + r * NS, es)] = a[r];
      }
    }
  }
  if constexpr (!LAST) {
    lds_sync<WAVE>();
    if (active) {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = lds[lds_at<PAD>(t + T * e, es)];
    }
    lds_sync<WAVE>();
  }
}

template <int N, int T, int DIR, bool WAVE, int PAD, bool DTW, int NS, int R, int... Rest>
__device__ __forceinline__ void stages(float2* v, float2* lds, int es, int t, bool active,
                                       const float2* __restrict__ tw) {
  constexpr bool last = sizeof...(Rest) == 0;
  stage<N, T, R, NS, DIR, last, WAVE, PAD, DTW>(v, lds, es, t, active, tw);
  if constexpr (!last) stages<N, T, DIR, WAVE, PAD, DTW, NS * R, Rest...>(v, lds, es, t, active, tw);
}

// Full length-N transform of the pencil held in v (cyclic in and out).
// DIR = +1: sum x_j exp(-2 pi i jk/N); DIR = -1: sum x_j exp(+2 pi i jk/N).
// Every thread of the block must call this (it contains barriers); `active`
// masks LDS traffic of threads without a pencil.
template <int N, int T, int DIR, int... Rs>
__device__ __forceinline__ void fft(float2* v, float2* lds, int es, int t, bool active,
                                    const float2* __restrict__ tw, Radices<Rs...>) {
  stages<N, T, DIR, false, 0, false, 1, Rs...>(v, lds, es, t, active, tw);
}
// the same with wavefront-scope ordering (every pencil inside one wavefront) and
// an optional padded LDS layout (lds_at)
template <int N, int T, int DIR, int PAD = 0, int... Rs>
__device__ __forceinline__ void fft_wave(float2* v, float2* lds, int es, int t, bool active,
                                         const float2* __restrict__ tw, Radices<Rs...>) {
  stages<N, T, DIR, true, PAD, false, 1, Rs...>(v, lds, es, t, active, tw);
}
// variants that read every twiddle W^(r k) directly from the table instead of
// forming it from the power-of-two entries: for tables staged in LDS, where a read
// costs less than the complex products it replaces
template <int N, int T, int DIR, int... Rs>
__device__ __forceinline__ void fft_dtw(float2* v, float2* lds, int es, int t, bool active,
                                        const float2* __restrict__ tw, Radices<Rs...>) {
  stages<N, T, DIR, false, 0, true, 1, Rs...>(v, lds, es, t, active, tw);
}
template <int N, int T, int DIR, int PAD = 0, int... Rs>
__device__ __forceinline__ void fft_wave_dtw(float2* v, float2* lds, int es, int t, bool active,
                                             const float2* __restrict__ tw, Radices<Rs...>) {
  stages<N, T, DIR, true, PAD, true, 1, Rs...>(v, lds, es, t, active, tw);
}

}  // namespace hmcfft

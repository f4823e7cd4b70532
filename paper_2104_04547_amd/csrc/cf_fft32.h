// 32-point complex FFT held in registers (one transform per thread), the building
// block of the frequency-domain 3-D convolution.
//
// Convention: forward X[k] = sum_n x[n] e^{-2 pi i n k / 32}; inverse (INV = true)
// x[n] = sum_k X[k] e^{+2 pi i n k / 32}, unnormalised.  Radix-2 decimation in
// time over bit-reversed inputs; every index is a compile-time constant once the
// loops unroll, so the arrays stay in VGPRs and the twiddles become immediates.
#pragma once

namespace cf {

// cos and sin of 2 pi t / 32 for t = 0 .. 15
constexpr float kFftCos32[16] = {1.000000000e+00f,  9.807852804e-01f,  9.238795325e-01f,  8.314696123e-01f,
                                 7.071067812e-01f,  5.555702330e-01f,  3.826834324e-01f,  1.950903220e-01f,
                                 0.0f,              -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
                                 -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f};
constexpr float kFftSin32[16] = {0.0f,             1.950903220e-01f, 3.826834324e-01f, 5.555702330e-01f,
                                 7.071067812e-01f, 8.314696123e-01f, 9.238795325e-01f, 9.807852804e-01f,
                                 1.000000000e+00f, 9.807852804e-01f, 9.238795325e-01f, 8.314696123e-01f,
                                 7.071067812e-01f, 5.555702330e-01f, 3.826834324e-01f, 1.950903220e-01f};

__host__ __device__ constexpr int fft_brev5(int i) {
  return ((i & 1) << 4) | ((i & 2) << 2) | (i & 4) | ((i & 8) >> 2) | ((i & 16) >> 4);
}

template <bool INV>
__host__ __device__ inline void fft32(float (&re)[32], float (&im)[32]) {
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int j = fft_brev5(i);
    if (j > i) {
      const float tr = re[i], ti = im[i];
      re[i] = re[j];
      im[i] = im[j];
      re[j] = tr;
      im[j] = ti;
    }
  }
#pragma unroll
  for (int half = 1; half < 32; half <<= 1) {
#pragma unroll
    for (int i = 0; i < 32; i += 2 * half) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int t = j * (16 / half);  // twiddle e^{-+2 pi i t / 32}
        const int a = i + j, b = i + j + half;
        float br, bi;
        if (t == 0) {
          br = re[b];
          bi = im[b];
        } else if (t == 8) {  // times -i (forward) or +i (inverse)
          br = INV ? -im[b] : im[b];
          bi = INV ? re[b] : -re[b];
        } else {
          const float c = kFftCos32[t], s = INV ? kFftSin32[t] : -kFftSin32[t];
          br = re[b] * c - im[b] * s;
          bi = re[b] * s + im[b] * c;
        }
        re[b] = re[a] - br;
        im[b] = im[a] - bi;
        re[a] = re[a] + br;
        im[a] = im[a] + bi;
      }
    }
  }
}

// 16-point complex FFT in registers (same conventions; twiddles e^{-+2 pi i 2t / 32})
template <bool INV>
__host__ __device__ inline void fft16(float (&re)[16], float (&im)[16]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int j = ((i & 1) << 3) | ((i & 2) << 1) | ((i & 4) >> 1) | ((i & 8) >> 3);
    if (j > i) {
      const float tr = re[i], ti = im[i];
      re[i] = re[j];
      im[i] = im[j];
      re[j] = tr;
      im[j] = ti;
    }
  }
#pragma unroll
  for (int half = 1; half < 16; half <<= 1) {
#pragma unroll
    for (int i = 0; i < 16; i += 2 * half) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const int t = 2 * j * (8 / half);  // twiddle e^{-+2 pi i t / 32}
        const int a = i + j, b = i + j + half;
        float br, bi;
        if (t == 0) {
          br = re[b];
          bi = im[b];
        } else if (t == 8) {
          br = INV ? -im[b] : im[b];
          bi = INV ? re[b] : -re[b];
        } else {
          const float c = kFftCos32[t], s = INV ? kFftSin32[t] : -kFftSin32[t];
          br = re[b] * c - im[b] * s;
          bi = re[b] * s + im[b] * c;
        }
        re[b] = re[a] - br;
        im[b] = im[a] - bi;
        re[a] = re[a] + br;
        im[a] = im[a] + bi;
      }
    }
  }
}

// value times e^{-+2 pi i t / 32}, t = 0 .. 15
template <bool INV>
__host__ __device__ inline void twiddle32(float &r, float &i, int t) {
  const float c = kFftCos32[t], s = INV ? kFftSin32[t] : -kFftSin32[t];
  const float nr = r * c - i * s, ni = r * s + i * c;
  r = nr;
  i = ni;
}

// A 32-point transform shared by two threads (h = 0, 1), each holding 16 points;
// `partner(v)` returns the other thread's value of v.
//
// Decimation in time: thread h holds x[2n + h] and ends with X[16 h + k], k = 0..15
// (each half-transform is a 16-point FFT; the odd half is twisted by e^{-+2 pi i k/32}
// and the two are combined as X[k] = E[k] + W^k O[k], X[k + 16] = E[k] - W^k O[k]).
template <bool INV, typename Partner>
__host__ __device__ inline void fft32_pair_dit(float (&re)[16], float (&im)[16], int h, Partner partner) {
  fft16<INV>(re, im);
  if (h) {
#pragma unroll
    for (int k = 1; k < 16; ++k) twiddle32<INV>(re[k], im[k], k);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float pr = partner(re[k]), pi = partner(im[k]);
    re[k] = h ? pr - re[k] : re[k] + pr;
    im[k] = h ? pi - im[k] : im[k] + pi;
  }
}

// Decimation in frequency: thread h holds x[16 h + n] and ends with X[2k + h]
// (X[2k] is the 16-point FFT of x[n] + x[n + 16], X[2k + 1] that of
// (x[n] - x[n + 16]) e^{-+2 pi i n / 32}).
template <bool INV, typename Partner>
__host__ __device__ inline void fft32_pair_dif(float (&re)[16], float (&im)[16], int h, Partner partner) {
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    const float pr = partner(re[n]), pi = partner(im[n]);
    re[n] = h ? pr - re[n] : re[n] + pr;
    im[n] = h ? pi - im[n] : im[n] + pi;
  }
  if (h) {
#pragma unroll
    for (int n = 1; n < 16; ++n) twiddle32<INV>(re[n], im[n], n);
  }
  fft16<INV>(re, im);
}

}  // namespace cf

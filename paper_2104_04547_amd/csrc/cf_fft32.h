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

}  // namespace cf

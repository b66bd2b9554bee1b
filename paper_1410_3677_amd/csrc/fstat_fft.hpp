// Device building blocks: complex arithmetic and an LDS-resident Stockham FFT
// for gfx950 (64-wide wavefronts).
//
// A workgroup transforms NC independent columns of LEN points that sit in LDS
// with a column stride STRIDE.  Each stage of radix R (8 while at least 8
// points remain, then 4 or 2) loads R points per butterfly into registers,
// applies the inter-stage twiddles, does an R-point DFT in registers, and
// writes the outputs back in Stockham (self-sorting) order, so the result is
// in natural order without a bit-reversal pass.
#pragma once

#include <hip/hip_runtime.h>

namespace fstat {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T re, T im) {
  cx<T> r;
  r.re = re;
  r.im = im;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.re * s, a.im * s); }
template <typename T>
__device__ __forceinline__ T cnorm2(cx<T> a) { return a.re * a.re + a.im * a.im; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return INV ? mk<T>(-a.im, a.re) : mk<T>(a.im, -a.re);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
  cx<T> s13 = v[1] + v[3], d13 = mul_mi<T, INV>(v[1] - v[3]);
  v[0] = s02 + s13;
  v[2] = s02 - s13;
  v[1] = d02 + d13;
  v[3] = d02 - d13;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  const T h = (T)0.70710678118654752440084436210485;
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  // o[k] *= W8^k, W8 = exp(-+ i pi/4)
  cx<T> o1 = INV ? mk<T>(h * (o[1].re - o[1].im), h * (o[1].re + o[1].im))
                 : mk<T>(h * (o[1].re + o[1].im), h * (o[1].im - o[1].re));
  cx<T> o2 = mul_mi<T, INV>(o[2]);
  cx<T> o3 = INV ? mk<T>(-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im))
                 : mk<T>(h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im));
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + o1;
  v[5] = e[1] - o1;
  v[2] = e[2] + o2;
  v[6] = e[2] - o2;
  v[3] = e[3] + o3;
  v[7] = e[3] - o3;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftr(cx<T>* v) {
  if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft2<T, INV>(v);
}

// One Stockham stage over NC columns of LEN points (column stride STRIDE),
// radix R, NS = product of the previous radices.  tw1024[m] = exp(-2 pi i m/1024).
template <typename T, int LEN, int NC, int NT, int STRIDE, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_stage(cx<T>* lds, const cx<T>* __restrict__ tw1024) {
  constexpr int NB = LEN / R;           // butterflies per column
  constexpr int TOT = NC * NB;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int TWSTEP = 1024 / (NS * R);
  const int tid = threadIdx.x;
  cx<T> v[PER][R];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if ((TOT % NT == 0) || b < TOT) {
      const int c = b / NB, j = b % NB;
      const cx<T>* col = lds + c * STRIDE;
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cx<T> x = col[j + r * NB];
        if (NS > 1 && r > 0) {
          cx<T> w = tw1024[k * r * TWSTEP];
          if (INV) w.im = -w.im;
          x = cmul(x, w);
        }
        v[i][r] = x;
      }
      dftr<T, R, INV>(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if ((TOT % NT == 0) || b < TOT) {
      const int c = b / NB, j = b % NB;
      cx<T>* col = lds + c * STRIDE;
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) col[base + r * NS] = v[i][r];
    }
  }
  __syncthreads();
}

template <typename T, int LEN, int NC, int NT, int STRIDE, bool INV, int NS>
__device__ __forceinline__ void lds_fft_from(cx<T>* lds, const cx<T>* __restrict__ tw1024) {
  if constexpr (NS < LEN) {
    constexpr int REM = LEN / NS;
    constexpr int R = REM >= 8 ? 8 : REM;
    stockham_stage<T, LEN, NC, NT, STRIDE, R, NS, INV>(lds, tw1024);
    lds_fft_from<T, LEN, NC, NT, STRIDE, INV, NS * R>(lds, tw1024);
  }
}

// In-place DFT (unnormalised; forward sign -i, INV sign +i) of NC LDS columns.
// Callers must __syncthreads() after filling LDS; the routine ends with a barrier.
template <typename T, int LEN, int NC, int NT, int STRIDE, bool INV>
__device__ __forceinline__ void lds_fft(cx<T>* lds, const cx<T>* __restrict__ tw1024) {
  static_assert(LEN >= 2 && LEN <= 1024 && (LEN & (LEN - 1)) == 0, "LEN must be a power of two <= 1024");
  lds_fft_from<T, LEN, NC, NT, STRIDE, INV, 1>(lds, tw1024);
}

// exp(-+ 2 pi i m / L) for 0 <= m < L from a split table: lo[m % 1024] * hi[m / 1024],
// lo[i] = W_L^i (i < 1024), hi[i] = W_L^(1024 i) (i < L/1024).
template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle_L(const cx<T>* __restrict__ lo, const cx<T>* __restrict__ hi, int m) {
  cx<T> w = cmul(lo[m & 1023], hi[m >> 10]);
  if (INV) w.im = -w.im;
  return w;
}

}  // namespace fstat

// HIP kernels of the F-statistic search path for gfx950.
//
// Per sky position (amortised over the spindown loop, Sect. 2):
//   k_sky_setup     direction, amplitude-modulation coefficients, n.r_0
//   k_sky_demod     a(t), b(t), Roemer delay, phase demodulation -> za, zb;
//                   per-block partial sums of a^2, b^2, ab (FP64)
//   k_sky_finalize  A, B, C in a fixed summation order and the 2F coefficients
//   k_fft_pass_a / k_fft_pass_b   2x upsampling by spectral zero-padding
//                   (forward length nfft/2, inverse length nfft)
//   k_spline        natural cubic spline through the upsampled series,
//                   evaluated at the detector positions of the barycentric grid
// Per (sky, spindown) template (the hot loop):
//   k_tmpl_pass_a   spindown chirp fused into the load, column DFTs of the
//                   four-step FFT, inter-pass twiddle
//   k_tmpl_pass_b   row DFTs, 2F for both amplitude series, threshold and
//                   stream compaction (or a store of the 2F spectrum)
//
// An nfft = P*Q point FFT is done in two passes over a P x Q view
// (j = j1 + P j2, k = Q k1 + k2):
//   pass A: for each column j1, Q-point DFT over j2, times W_nfft^(j1 k2),
//           stored transposed as T[k2][j1];
//   pass B: for each row k2, P-point DFT over j1 -> X[Q k1 + k2].
// Each workgroup handles TW adjacent columns (pass A) or rows (pass B) of both
// amplitude series, so global loads and stores move TW contiguous elements.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fstat_fft.hpp"

namespace fstat {

constexpr int NT = 256;  // threads per workgroup (4 wavefronts)

// Earth rotation rate: 2 pi / sidereal day (86164.0905 s).
__host__ __device__ constexpr double sidereal_rate() { return 6.283185307179586476925 / 86164.0905; }

struct SkyParams {
  double nx, ny, nz;           // unit vector towards the source
  double nr0;                  // n . r_0
  double x0;                   // alpha - phi_r
  double ka[5];                // a = ka0 cos2x + ka1 sin2x + ka2 cos x + ka3 sin x + ka4
  double kb[4];                // b = kb0 cos2x + kb1 sin2x + kb2 cos x + kb3 sin x
  double A, B, C;              // <a^2>, <b^2>, <ab>
  double cfa, cfb, cfab;       // 2F = cfa |Fa|^2 + cfb |Fb|^2 + cfab Re(Fa Fb*)
  double pad[2];
};

struct SegConst {
  int n;            // samples
  int nfft;         // L
  double dt, f_off, sigma2;
  double lat, gamma, phi_r;
  const double* x;  // n
  const double* r;  // 3 n, component-major
};

// Candidate entry as written by the threshold stage.
struct CandEntry {
  int32_t search, segment, sky, fdot_idx, bin, pad;
  double twoF;
};

// ------------------------------------------------------------------ sky stage
__global__ void k_sky_setup(const double* __restrict__ alpha, const double* __restrict__ delta,
                            int sky0, int nsky, SegConst sc, SkyParams* __restrict__ sp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsky) return;
  const double al = alpha[sky0 + i], de = delta[sky0 + i];
  double sa, ca, sd, cd;
  sincos(al, &sa, &ca);
  sincos(de, &sd, &cd);
  SkyParams p;
  p.nx = cd * ca;
  p.ny = cd * sa;
  p.nz = sd;
  p.nr0 = p.nx * sc.r[0] + p.ny * sc.r[sc.n] + p.nz * sc.r[2 * sc.n];
  p.x0 = al - sc.phi_r;
  double s2g, c2g, sl, cl, s2l, c2l;
  sincos(2.0 * sc.gamma, &s2g, &c2g);
  sincos(sc.lat, &sl, &cl);
  sincos(2.0 * sc.lat, &s2l, &c2l);
  const double s2d = 2.0 * sd * cd, c2d = cd * cd - sd * sd;
  p.ka[0] = s2g * (3.0 - c2l) * (3.0 - c2d) / 16.0;
  p.ka[1] = -c2g * sl * (3.0 - c2d) / 4.0;
  p.ka[2] = s2g * s2l * s2d / 4.0;
  p.ka[3] = -c2g * cl * s2d / 2.0;
  p.ka[4] = 0.75 * s2g * cl * cl * cd * cd;
  p.kb[0] = c2g * sl * sd;
  p.kb[1] = s2g * (3.0 - c2l) * sd / 4.0;
  p.kb[2] = c2g * cl * cd;
  p.kb[3] = s2g * s2l * cd / 2.0;
  p.A = p.B = p.C = 0.0;
  p.cfa = p.cfb = p.cfab = 0.0;
  p.pad[0] = p.pad[1] = 0.0;
  sp[i] = p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Demodulation: za = x a e^{-i psi}, zb = x b e^{-i psi}, psi = 2 pi f_off D (reduced mod 2 pi
// in FP64).  za/zb of sky i, series s at zab + (2 i + s) * ldz.  Partial sums of a^2, b^2, ab
// per block at part[(i * gridDim.x + blockIdx.x) * 3 + c].
template <typename T>
__global__ void __launch_bounds__(NT) k_sky_demod(SegConst sc, const SkyParams* __restrict__ sp,
                                                  cx<T>* __restrict__ zab, long ldz, double* __restrict__ part) {
  const int i = blockIdx.y;
  const SkyParams p = sp[i];
  const int j = blockIdx.x * NT + threadIdx.x;
  double aa = 0.0, bb = 0.0, ab = 0.0;
  if (j < sc.n) {
    const double t = (double)j * sc.dt;
    double sx, cx_;
    sincos(p.x0 - sidereal_rate() * t, &sx, &cx_);
    const double c2x = cx_ * cx_ - sx * sx, s2x = 2.0 * sx * cx_;
    const double a = p.ka[0] * c2x + p.ka[1] * s2x + p.ka[2] * cx_ + p.ka[3] * sx + p.ka[4];
    const double b = p.kb[0] * c2x + p.kb[1] * s2x + p.kb[2] * cx_ + p.kb[3] * sx;
    const double d = p.nx * sc.r[j] + p.ny * sc.r[sc.n + j] + p.nz * sc.r[2 * sc.n + j] - p.nr0;
    double cyc = sc.f_off * d;
    cyc -= floor(cyc);
    T s, c;
    if constexpr (sizeof(T) == 8) {
      sincospi(2.0 * cyc, &s, &c);
    } else {
      sincospif((float)(2.0 * cyc), &s, &c);
    }
    const double xa = sc.x[j] * a, xb = sc.x[j] * b;
    zab[(2 * i) * ldz + j] = mk<T>((T)xa * c, -(T)xa * s);
    zab[(2 * i + 1) * ldz + j] = mk<T>((T)xb * c, -(T)xb * s);
    aa = a * a;
    bb = b * b;
    ab = a * b;
  }
  __shared__ double red[3][NT / 64];
  aa = wave_sum(aa);
  bb = wave_sum(bb);
  ab = wave_sum(ab);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = aa;
    red[1][w] = bb;
    red[2][w] = ab;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) v += red[threadIdx.x][k];
    part[((long)i * gridDim.x + blockIdx.x) * 3 + threadIdx.x] = v;
  }
}

// A, B, C and the 2F coefficients of each sky (one workgroup per sky, fixed order).
__global__ void __launch_bounds__(NT) k_sky_finalize(SegConst sc, SkyParams* __restrict__ sp,
                                                     const double* __restrict__ part, int nblk, int full_form) {
  const int i = blockIdx.x;
  double s[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += NT)
    for (int c = 0; c < 3; ++c) s[c] += part[((long)i * nblk + b) * 3 + c];
  __shared__ double red[3][NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = 0; c < 3; ++c) {
    double v = wave_sum(s[c]);
    if (lane == 0) red[c][w] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[3];
    for (int c = 0; c < 3; ++c) {
      t[c] = 0.0;
      for (int k = 0; k < NT / 64; ++k) t[c] += red[c][k];
    }
    SkyParams& p = sp[i];
    p.A = t[0] / sc.n;
    p.B = t[1] / sc.n;
    p.C = t[2] / sc.n;
    const double norm = 2.0 / ((double)sc.n * sc.sigma2);
    if (full_form) {
      const double D = p.A * p.B - p.C * p.C;
      p.cfa = norm * p.B / D;
      p.cfb = norm * p.A / D;
      p.cfab = -2.0 * norm * p.C / D;
    } else {
      p.cfa = norm / p.A;
      p.cfb = norm / p.B;
      p.cfab = 0.0;
    }
  }
}

// ------------------------------------------------------------ generic FFT passes
// Column stride of an LDS tile: LEN plus one element breaks power-of-two strides.
template <int LEN>
constexpr int lds_stride() { return LEN + 1; }

// Workgroup tile width: columns per workgroup so that both series fit in 64 KiB of LDS.
template <typename T, int LEN>
constexpr int tile_width() {
  constexpr int tw = (64 * 1024) / (2 * (int)sizeof(cx<T>) * (LEN + 1));
  constexpr int p2 = tw >= 16 ? 16 : tw >= 8 ? 8 : tw >= 4 ? 4 : tw >= 2 ? 2 : 1;
  return p2;
}

enum SrcKind { SRC_PLAIN = 0, SRC_HALFSHIFT = 1 };

// Map a linear workgroup id to (tile, item) so that each XCD (workgroups are
// dealt round-robin over 8 XCDs) keeps a fixed subset of tiles for all items.
__device__ __forceinline__ void xcd_tile_item(int ntiles, int& tile, int& item) {
  const int b = blockIdx.x;
  if ((ntiles & 7) == 0) {
    const int per = ntiles >> 3;
    const int xcd = b & 7, r = b >> 3;
    tile = xcd * per + (r % per);
    item = r / per;
  } else {
    tile = b % ntiles;
    item = b / ntiles;
  }
}

// Pass A of an L = P*Q FFT (DFT length Q along j2), two series per item.
//   SRC_PLAIN:     x_s[j] = in[(2 item + s) * ld_in + j] for j < nvalid, else 0
//   SRC_HALFSHIFT: x_s[k] = Z[k] exp(i pi k_s / L), k_s = k for k < L/2, k - L otherwise
//                  (Z = in, the spectrum of a series of L samples; shlo, shhi: the
//                  twiddle tables of length 2L).  The inverse transform of x is the
//                  series half a sample later, the odd samples of its band-limited 2x
//                  upsampling with the Nyquist term on the negative side.
// Output T_s[k2 * P + j1] at out + (2 item + s) * L.
template <typename T, int Q, bool INV, int SRC>
__global__ void __launch_bounds__(NT) k_fft_pass_a(const cx<T>* __restrict__ in, long ld_in, int nvalid,
                                                   cx<T>* __restrict__ out, int P, int L,
                                                   const cx<T>* __restrict__ tw1024,
                                                   const cx<T>* __restrict__ twlo, const cx<T>* __restrict__ twhi,
                                                   const cx<T>* __restrict__ shlo, const cx<T>* __restrict__ shhi) {
  constexpr int TW = tile_width<T, Q>();
  constexpr int ST = lds_stride<Q>();
  __shared__ cx<T> lds[2 * TW * ST];
  int tile, item;
  xcd_tile_item(P / TW, tile, item);
  const int j10 = tile * TW;
  for (int e = threadIdx.x; e < 2 * TW * Q; e += NT) {
    const int s = e / (TW * Q), rem = e % (TW * Q);
    const int j2 = rem / TW, c = rem % TW;
    const int j = j10 + c + P * j2;
    cx<T> v = mk<T>(0, 0);
    const cx<T>* src = in + (2 * item + s) * ld_in;
    if (SRC == SRC_PLAIN) {
      if (j < nvalid) v = src[j];
    } else {
      cx<T> w = twiddle_L<T, true>(shlo, shhi, j);
      if (j >= (L >> 1)) w = mk<T>(-w.re, -w.im);
      v = cmul(src[j], w);
    }
    lds[(s * TW + c) * ST + j2] = v;
  }
  __syncthreads();
  lds_fft<T, Q, 2 * TW, NT, ST, INV>(lds, tw1024);
  for (int e = threadIdx.x; e < 2 * TW * Q; e += NT) {
    const int s = e / (TW * Q), rem = e % (TW * Q);
    const int k2 = rem / TW, c = rem % TW;
    const int j1 = j10 + c;
    cx<T> v = cmul(lds[(s * TW + c) * ST + k2], twiddle_L<T, INV>(twlo, twhi, j1 * k2));
    out[(long)(2 * item + s) * L + (long)k2 * P + j1] = v;
  }
}

// Pass B of an L = P*Q FFT (DFT length P along j1) with natural-order output:
// X_s[Q k1 + k2] * scale at out + (2 item + s) * ld_out.
template <typename T, int P, bool INV>
__global__ void __launch_bounds__(NT) k_fft_pass_b(const cx<T>* __restrict__ in, cx<T>* __restrict__ out,
                                                   long ld_out, int Q, int L, T scale,
                                                   const cx<T>* __restrict__ tw1024) {
  constexpr int TW = tile_width<T, P>();
  constexpr int ST = lds_stride<P>();
  __shared__ cx<T> lds[2 * TW * ST];
  int tile, item;
  xcd_tile_item(Q / TW, tile, item);
  const int k20 = tile * TW;
  for (int e = threadIdx.x; e < 2 * TW * P; e += NT) {
    const int s = e / (TW * P), rem = e % (TW * P);
    const int c = rem / P, j1 = rem % P;
    lds[(s * TW + c) * ST + j1] = in[(long)(2 * item + s) * L + (long)(k20 + c) * P + j1];
  }
  __syncthreads();
  lds_fft<T, P, 2 * TW, NT, ST, INV>(lds, tw1024);
  for (int e = threadIdx.x; e < 2 * TW * P; e += NT) {
    const int s = e / (TW * P), rem = e % (TW * P);
    const int k1 = rem / TW, c = rem % TW;
    out[(long)(2 * item + s) * ld_out + (long)Q * k1 + k20 + c] = cscale(lds[(s * TW + c) * ST + k1], scale);
  }
}

// ----------------------------------------------------------------- resampling
// Sample q of the 2x upsampled series: the even samples are the series z itself (zero
// from n on), the odd samples the series o half a sample later.
template <typename T>
__device__ __forceinline__ cx<T> upsampled(const cx<T>* __restrict__ z, const cx<T>* __restrict__ o, int q, int n) {
  const int h = q >> 1;
  if (q & 1) return o[h];
  return h < n ? z[h] : mk<T>(0, 0);
}

// The 2x upsampled series of a batch of skies, for stage-by-stage checks: u[q] of each
// series of z and o (stride ldz) into out (stride L).
template <typename T>
__global__ void __launch_bounds__(NT) k_upsampled(const cx<T>* __restrict__ z, const cx<T>* __restrict__ o,
                                                  long ldz, int n, int L, cx<T>* __restrict__ out) {
  const int q = blockIdx.x * NT + threadIdx.x, s = blockIdx.y;
  if (q < L) out[(long)s * L + q] = upsampled(z + s * ldz, o + s * ldz, q, n);
}
// Natural cubic spline through the upsampled series u[0..L) (unit spacing),
// evaluated at 2 s_j with s_j = j - D_j/dt; zero where s_j is outside [0, n-1].
// Spline moments: m_0 = m_{L-1} = 0, m_{p-1} + 4 m_p + m_{p+1} = d_p = 6 (u_{p+1} - 2u_p + u_{p-1}).
// They are computed as m_p = sum_q G(p, q) d_q with the Green's function of the
// (1, 4, 1) operator, g(k) = z^|k| / (2 sqrt 3), z = sqrt 3 - 2, and odd images at
// both ends: G(p, q) = g(p-q) - g(p+q) - g(2(L-1)-p-q), truncated at |k| <= KT
// (|z|^KT below the working precision).
template <typename T, int KT>
__device__ __forceinline__ cx<T> spline_moment(int p, int L, const cx<T>* d, int dlo, const T* g,
                                               const T* __restrict__ gg) {
  // d[q - dlo] = d_q for q in [max(1, p - KT), min(L - 2, p + KT)]
  if (p <= 0 || p >= L - 1) return mk<T>(0, 0);
  if (p > KT && p < L - 1 - KT) {
    // interior knot: no image terms, the symmetric 2 KT + 1 taps with the weights read as
    // uniform values (gg: the same table in global memory)
    const cx<T>* c = d + (p - dlo);
    cx<T> acc = mk<T>(gg[0] * c[0].re, gg[0] * c[0].im);
#pragma unroll
    for (int k = 1; k <= KT; ++k) {
      const cx<T> a = c[-k], b = c[k];
      acc = mk<T>(acc.re + gg[k] * (a.re + b.re), acc.im + gg[k] * (a.im + b.im));
    }
    return acc;
  }
  cx<T> acc = mk<T>(0, 0);
  const int q0 = max(1, p - KT), q1 = min(L - 2, p + KT);
  for (int q = q0; q <= q1; ++q) {
    const int dpq = p > q ? p - q : q - p;
    T w = g[dpq];
    if (p + q <= KT) w -= g[p + q];
    const int far = 2 * (L - 1) - p - q;
    if (far <= KT) w -= g[far];
    const cx<T> dq = d[q - dlo];
    acc = mk<T>(acc.re + w * dq.re, acc.im + w * dq.im);
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ cx<T> spline_eval(cx<T> u0, cx<T> u1, cx<T> m0, cx<T> m1, T t) {
  const T w = (T)1 - t;
  const T c0 = (w * w * w - w) / (T)6, c1 = (t * t * t - t) / (T)6;
  return mk<T>(w * u0.re + t * u1.re + c0 * m0.re + c1 * m1.re,
               w * u0.im + t * u1.im + c0 * m0.im + c1 * m1.im);
}

// u of sky i, series s at u + (2 i + s) * L; output zt + (2 i + s) * ldzt.
// One workgroup covers NT outputs j; their knot range [pmin, pmax + 1] is staged in
// LDS together with the curvature sources d_q within KT of it.
template <typename T, int KT>
__global__ void __launch_bounds__(NT) k_spline(SegConst sc, const SkyParams* __restrict__ sp,
                                               const cx<T>* __restrict__ z, const cx<T>* __restrict__ o, long ldz,
                                               cx<T>* __restrict__ zt, long ldzt, const T* __restrict__ gtab) {
  constexpr int CAP = 2 * NT + 64;              // knots held for one tile
  constexpr int DCAP = CAP + 2 * KT + 2;        // curvature sources held
  __shared__ cx<T> su[2][DCAP + 2];
  __shared__ cx<T> sd[2][DCAP];
  __shared__ cx<T> sm[2][CAP + 1];
  __shared__ T sg[KT + 1];
  __shared__ int sminmax[2];
  const int i = blockIdx.y;
  const int L = sc.nfft, n = sc.n;
  const SkyParams p = sp[i];
  const int j = blockIdx.x * NT + threadIdx.x;
  bool valid = false;
  int kn = 0;
  T tf = 0;
  if (j < n) {
    const double d = p.nx * sc.r[j] + p.ny * sc.r[n + j] + p.nz * sc.r[2 * n + j] - p.nr0;
    const double s = (double)j - d / sc.dt;
    valid = (s >= 0.0) && (s <= (double)(n - 1));
    if (valid) {
      const double pos = 2.0 * s;
      kn = (int)floor(pos);
      kn = min(max(kn, 0), L - 2);
      tf = (T)(pos - (double)kn);
    }
  }
  if (threadIdx.x <= KT) sg[threadIdx.x] = gtab[threadIdx.x];
  if (threadIdx.x == 0) {
    sminmax[0] = 0x7fffffff;
    sminmax[1] = -1;
  }
  __syncthreads();
  {
    // the tile's knot range: a wavefront reduction, then one LDS atomic per wavefront
    int mn = valid ? kn : 0x7fffffff, mx = valid ? kn : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mn = min(mn, __shfl_xor(mn, off, 64));
      mx = max(mx, __shfl_xor(mx, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
      atomicMin(&sminmax[0], mn);
      atomicMax(&sminmax[1], mx);
    }
  }
  __syncthreads();
  const int pmin = sminmax[0], pmax = sminmax[1];
  if (pmax < 0) {  // no valid output in this tile
    if (j < n) {
      zt[(2 * i) * ldzt + j] = mk<T>(0, 0);
      zt[(2 * i + 1) * ldzt + j] = mk<T>(0, 0);
    }
    return;
  }
  const cx<T>* za = z + (long)(2 * i) * ldz;
  const cx<T>* zb = z + (long)(2 * i + 1) * ldz;
  const cx<T>* oa = o + (long)(2 * i) * ldz;
  const cx<T>* ob = o + (long)(2 * i + 1) * ldz;
  if (pmax + 1 - pmin + 1 <= CAP) {
    // knots needed for moments [pmin, pmax+1]: sources q in [pmin-KT, pmax+1+KT], each uses u[q-1..q+1]
    const int dlo = max(1, pmin - KT), dhi = min(L - 2, pmax + 1 + KT);
    const int ulo = dlo - 1, uhi = dhi + 1;
    for (int q = ulo + threadIdx.x; q <= uhi; q += NT) {
      su[0][q - ulo] = upsampled(za, oa, q, n);
      su[1][q - ulo] = upsampled(zb, ob, q, n);
    }
    __syncthreads();
    for (int q = dlo + threadIdx.x; q <= dhi; q += NT) {
      for (int s = 0; s < 2; ++s) {
        const cx<T> a = su[s][q - 1 - ulo], b = su[s][q - ulo], c = su[s][q + 1 - ulo];
        sd[s][q - dlo] = mk<T>((T)6 * (c.re - (T)2 * b.re + a.re), (T)6 * (c.im - (T)2 * b.im + a.im));
      }
    }
    __syncthreads();
    for (int q = pmin + threadIdx.x; q <= pmax + 1; q += NT) {
      sm[0][q - pmin] = spline_moment<T, KT>(q, L, sd[0], dlo, sg, gtab);
      sm[1][q - pmin] = spline_moment<T, KT>(q, L, sd[1], dlo, sg, gtab);
    }
    __syncthreads();
    if (j < n) {
      cx<T> va = mk<T>(0, 0), vb = mk<T>(0, 0);
      if (valid) {
        // pmin >= ulo + 1 and pmax + 1 <= uhi, so both knots are staged
        va = spline_eval(su[0][kn - ulo], su[0][kn + 1 - ulo], sm[0][kn - pmin], sm[0][kn + 1 - pmin], tf);
        vb = spline_eval(su[1][kn - ulo], su[1][kn + 1 - ulo], sm[1][kn - pmin], sm[1][kn + 1 - pmin], tf);
      }
      zt[(2 * i) * ldzt + j] = va;
      zt[(2 * i + 1) * ldzt + j] = vb;
    }
  } else {
    // wide knot range (irregular delays): every thread works from global memory
    if (j < n) {
      cx<T> out[2] = {mk<T>(0, 0), mk<T>(0, 0)};
      if (valid) {
        for (int s = 0; s < 2; ++s) {
          const cx<T>* zs = s ? zb : za;
          const cx<T>* os = s ? ob : oa;
          auto us = [&](int q) { return upsampled(zs, os, q, n); };
          cx<T> m01[2];
          for (int h = 0; h < 2; ++h) {
            const int pp = kn + h;
            cx<T> acc = mk<T>(0, 0);
            if (pp > 0 && pp < L - 1) {
              const int q0 = max(1, pp - KT), q1 = min(L - 2, pp + KT);
              for (int q = q0; q <= q1; ++q) {
                const cx<T> a = us(q - 1), b = us(q), c = us(q + 1);
                const cx<T> dq = mk<T>((T)6 * (c.re - (T)2 * b.re + a.re), (T)6 * (c.im - (T)2 * b.im + a.im));
                const int dpq = pp > q ? pp - q : q - pp;
                T w = sg[dpq];
                if (pp + q <= KT) w -= sg[pp + q];
                const int far = 2 * (L - 1) - pp - q;
                if (far <= KT) w -= sg[far];
                acc = mk<T>(acc.re + w * dq.re, acc.im + w * dq.im);
              }
            }
            m01[h] = acc;
          }
          out[s] = spline_eval(us(kn), us(kn + 1), m01[0], m01[1], tf);
        }
      }
      zt[(2 * i) * ldzt + j] = out[0];
      zt[(2 * i + 1) * ldzt + j] = out[1];
    }
  }
}

// ------------------------------------------------------------- template stage
struct TmplArgs {
  int n, P, Q, L;       // samples; template FFT L = P * Q
  float ibw;            // interbinning weight (second pass with interbinning only)
  int nfdot;            // spindowns per sky
  int t0;               // first template of this launch (within the sky batch)
  int sky0;             // global index of the batch's first sky
  double dt;
  const double* fdot;   // device list (explicit spindowns), or NULL on a lattice grid
  long ldzt;            // stride between series in zt
  // lattice grid (fdot NULL): template (sky, index) has spindown integer s = s_lo + index
  const double* w_freq; // per sky: w0 component of the sky vectors' combination
  const double* w_spin; // per sky: w1 component
  double m10, m11;      // w0 and w1 components of the spindown row
  double bins_per_rad;  // nfft / (2 pi)
  int s_lo, nfft;
};

// Lattice arithmetic shared by the kernels and the host's candidate records, with
// contraction off so that both round every product and sum the same way.
// s row + sky: a component of the grid point s M1 + (n M2 + m M3).
__host__ __device__ inline double lattice_w(int s, double row, double sky) {
#pragma clang fp contract(off)
  return (double)s * row + sky;
}

// Shift u, in bins of the nfft grid, of a template's frequencies above the Fourier bins:
// the fraction of w0 nfft / (2 pi) above the integer below it, where a value within 1e-6
// below an integer counts as that integer (u in [-1e-6, 1 - 1e-6)).
__host__ __device__ inline double lattice_shift_bins(double w0, double bins_per_rad) {
#pragma clang fp contract(off)
  const double x = w0 * bins_per_rad;
  return x - floor(x + 1e-6);
}

// Spindown chirp of one template in cycles, (c2 j + c1) j at resampled sample j:
// c2 = fdot dt^2 / 2 for an explicit spindown; on a lattice c2 = w1 / (2 pi) and
// c1 = u / nfft, the shift that puts the grid's frequencies on the transform's bins.
__device__ __forceinline__ void template_chirp(const TmplArgs& ta, int skyl, int sidx, double& c2, double& c1) {
  if (ta.fdot) {
    c2 = 0.5 * ta.fdot[sidx] * ta.dt * ta.dt;
    c1 = 0.0;
  } else {
    const int sky = ta.sky0 + skyl, s = ta.s_lo + sidx;
    c2 = lattice_w(s, ta.m11, ta.w_spin[sky]) * (0.5 / M_PI);
    c1 = lattice_shift_bins(lattice_w(s, ta.m10, ta.w_freq[sky]), ta.bins_per_rad) / (double)ta.nfft;
  }
}

// Where pass B puts its results.
struct OutArgs {
  int k_min, k_max;
  double threshold;
  const int* search_next;        // device: searches begun so far (this one included)
  int segment;
  CandEntry* cand;               // candidate buffer
  unsigned long long* count;     // crossings found so far (may exceed capacity)
  long long capacity;
  void* spectrum;                // [sky][fdot][k - k_min], T
};

// Start of a search: advance the device-side search index.
__global__ void k_begin_search(int* search_next) {
  if (threadIdx.x == 0 && blockIdx.x == 0) search_next[0] += 1;
}

// Exclusive prefix sum of one int per thread over a workgroup of NTH threads;
// returns the thread's offset and writes the total to *total (all threads).
template <int NTH>
__device__ __forceinline__ int block_exclusive_scan_n(int v, int* total) {
  __shared__ int wsum[NTH / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < NTH / 64; ++k) {
    const int ws = wsum[k];
    if (k < w) before += ws;
    all += ws;
  }
  *total = all;
  return before + x - v;
}

// ------------------------------------------------------------ lattice sky loop
struct LatSkyArgs {
  double r2x, r2y, r3x, r3y;   // sky components (w2, w3) of rows 2 and 3
  double r2f, r2s, r3f, r3s;   // their w0 and w1 components
  double w;                    // W = 2 pi f_ref (1 AU / c)
  double ce, se;               // cos, sin of the obliquity
  double hemi;                 // +1 or -1
  int n_lo, m_lo, mspan;       // box origin and its extent in m
  long long total, capacity;   // box points; output capacity
  double *alpha, *delta, *w_freq, *w_spin;
  int* nm;
  long long* count;
};

// Sky loop of the lattice grid: every (n, m) of the box whose point (w2, w3) lies on the
// sky's disk, numbered in (n, m) order and written at its number.  One workgroup walks
// the box 256 points at a time (a workgroup scan numbers the points of each step), so
// the order needs no device-wide synchronisation.  The on-sky test and the w components
// are rounded as plain IEEE products and sums (no contraction).
__global__ __launch_bounds__(256) void k_lattice_sky(LatSkyArgs a) {
  long long base = 0;
  for (long long i0 = 0; i0 < a.total; i0 += 256) {
    const long long i = i0 + threadIdx.x;
    int on = 0, n = 0, m = 0;
    double xe = 0.0, ye = 0.0, r2 = 0.0;
    if (i < a.total) {
      n = a.n_lo + (int)(i / a.mspan);
      m = a.m_lo + (int)(i % a.mspan);
      {
#pragma clang fp contract(off)
        const double w2 = (double)n * a.r2x + (double)m * a.r3x;
        const double w3 = (double)n * a.r2y + (double)m * a.r3y;
        xe = w2 / a.w;
        ye = w3 / a.w;
        r2 = xe * xe + ye * ye;
      }
      on = r2 <= 1.0 ? 1 : 0;
    }
    int total = 0;
    const long long k = base + block_exclusive_scan_n<256>(on, &total);
    if (on && k < a.capacity) {
      double ze, wf, ws;
      {
#pragma clang fp contract(off)
        ze = a.hemi * sqrt(1.0 - r2);
        wf = (double)n * a.r2f + (double)m * a.r3f;
        ws = (double)n * a.r2s + (double)m * a.r3s;
      }
      // ecliptic to equatorial axes: rotation by the obliquity about the x axis
      const double x = xe;
      const double y = a.ce * ye - a.se * ze;
      const double z = a.se * ye + a.ce * ze;
      double al = atan2(y, x);
      if (al < 0.0) al += 2.0 * M_PI;
      a.alpha[k] = al;
      a.delta[k] = asin(fmin(1.0, fmax(-1.0, z)));
      a.w_freq[k] = wf;
      a.w_spin[k] = ws;
      if (a.nm) {
        a.nm[2 * k] = n;
        a.nm[2 * k + 1] = m;
      }
    }
    base += total;
    __syncthreads();   // the scan's LDS is reused by the next step
  }
  if (threadIdx.x == 0) *a.count = base;
}

}  // namespace fstat

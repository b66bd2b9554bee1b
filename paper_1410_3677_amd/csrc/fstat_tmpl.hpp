// Per-template kernels of the hot loop (spindown chirp, two-pass FFT, 2F, threshold).
//
// An nfft = P*Q FFT of both amplitude series of a template, j = j1 + P j2, k = Q k1 + k2:
//   pass A  for each column j1: Q-point DFT over j2 of y[j1 + P j2] (the resampled
//           series times the spindown chirp, zero beyond n), times W_nfft^(j1 k2),
//           stored to the intermediate T[k2][j1];
//   pass B  for each row k2: P-point DFT over j1 of T[k2][.], giving Fa, Fb at
//           k = Q k1 + k2, then 2F, threshold and candidate compaction.
//
// Both passes run radix-8 Stockham stages with one butterfly group per thread.
// The first stage reads its eight inputs straight from global memory and the
// last stage hands its outputs straight to global memory (pass A) or to the
// F-statistic (pass B), so only the exchanges between stages go through LDS.
// LDS index i of a column is stored at i + i/8 and columns are spaced so that
// the 16 lanes served per LDS cycle hit distinct banks:
//   pass A lanes run fastest over columns (coalesced rows of the input and of T),
//   pass B lanes run fastest along a row.
#pragma once

#include "fstat_kernels.hpp"

namespace fstat {

__host__ __device__ constexpr int phys(int i) { return i + (i >> 3); }

// radix of the stage that starts at stride NS for a LEN-point transform
template <int LEN, int NS>
__host__ __device__ constexpr int stage_radix() {
  return (LEN / NS) >= 8 ? 8 : (LEN / NS);
}

// threads per first-pass workgroup: FP32 workgroups cover eight columns of 512-point and
// 256-point columns (one 128-byte (a, b) line per row: 512 threads for 512-point columns,
// 256 for 256-point ones, 0.39 against 0.42 us per 2^17-point template with 512);
// 512 threads otherwise
template <typename T, int Q>
__host__ __device__ constexpr int tmpl_nt_a() { return sizeof(T) == 4 ? (Q == 256 ? 256 : 512) : 256; }
// butterfly groups per column of LEN points (one radix-8 butterfly per thread and stage)
template <int LEN>
__host__ __device__ constexpr int groups_per_col() { return LEN / 8; }
// pass B: 256 threads, each row owned by one wavefront (or a fraction of one) when
// its butterfly groups fit in 64 lanes
template <typename T, int LEN>
__host__ __device__ constexpr int tmpl_nt_b() { return 256; }
template <int LEN>
__host__ __device__ constexpr bool rows_in_wave() { return groups_per_col<LEN>() <= 64; }

// LDS ordering between the stages of columns that one wavefront owns: a wavefront's
// LDS operations complete in order, so only compiler reordering must be prevented.
template <bool WAVE_ONLY>
__device__ __forceinline__ void stage_sync() {
  if constexpr (WAVE_ONLY) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}
template <typename T, int LEN>
__host__ __device__ constexpr int tw_a() { return tmpl_nt_a<T, LEN>() / groups_per_col<LEN>(); }
template <typename T, int LEN>
__host__ __device__ constexpr int tw_b() { return tmpl_nt_b<T, LEN>() / groups_per_col<LEN>(); }

// column stride: phys(LEN) rounded so that stride % 32 == want (in complex elements)
template <int LEN>
__host__ __device__ constexpr int col_stride(int want) {
  return phys(LEN) + ((want - (phys(LEN) % 32)) % 32 + 32) % 32;
}
template <int TW>
__host__ __device__ constexpr int want_a() { return TW >= 16 ? 1 : 16 / TW; }

// Stage twiddles exp(-2 pi i k r / (NS R)), k < NS, 1 <= r < R, stored per (NS, R) as
// [k][r - 1] so that one butterfly's R - 1 twiddles are adjacent.  Tables exist for
// NS in {8, 64, 512} and R in {2, 4, 8}; stage_tw_offset gives each table's start.
__host__ __device__ constexpr int stage_tw_offset(int NS, int R) {
  int off = 0;
  for (int ns = 8; ns <= 512; ns *= 8)
    for (int rr = 2; rr <= 8; rr *= 2) {
      if (ns == NS && rr == R) return off;
      off += ns * (rr - 1);
    }
  return -1;
}
constexpr int STAGE_TW_ENTRIES = 8 * 11 + 64 * 11 + 512 * 11;

template <typename T, int NS, int R, bool INV>
__device__ __forceinline__ cx<T> stage_tw(const cx<T>* __restrict__ twst, int k, int r) {
  constexpr int OFF = stage_tw_offset(NS, R);
  static_assert(OFF >= 0, "no twiddle table for this stage");
  cx<T> w = twst[OFF + k * (R - 1) + (r - 1)];
  if (INV) w.im = -w.im;
  return w;
}

// Loads of one stage for butterflies j = g + G*b (b < PB) from an LDS column, twiddled, DFT'd.
// R is the stage radix, PB = (LEN / R) / G the butterflies per thread.
template <typename T, int LEN, int G, int NS, int R, int PB, bool INV>
__device__ __forceinline__ void stage_from_lds(cx<T> (&v)[PB][R], const cx<T>* col, int g,
                                               const cx<T>* __restrict__ twst) {
  constexpr int NB = LEN / R;
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int j = g + G * b;
    const int k = j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cx<T> x = col[phys(j + r * NB)];
      if constexpr (NS > 1) {
        if (r > 0) x = cmul(x, stage_tw<T, NS, R, INV>(twst, k, r));
      }
      v[b][r] = x;
    }
    dftr<T, R, INV>(v[b]);
  }
}

template <typename T, int LEN, int G, int NS, int R, int PB>
__device__ __forceinline__ void stage_to_lds(const cx<T> (&v)[PB][R], cx<T>* col, int g) {
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int j = g + G * b;
    const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) col[phys(base + r * NS)] = v[b][r];
  }
}

// The same stage loads and stores addressed as one LDS base plus compile-time offsets:
// phys(a + c) = phys(a) + c + c/8 whenever c is a multiple of 8, or a % 8 + c < 8.
template <typename T, int LEN, int G, int NS, int R, int PB, bool INV>
__device__ __forceinline__ void stage_from_lds_off(cx<T> (&v)[PB][R], const cx<T>* col, int g,
                                                   const cx<T>* __restrict__ twst) {
  constexpr int NB = LEN / R;
  static_assert(NB % 8 == 0 && (PB == 1 || G % 8 == 0), "constant offsets need multiples of 8");
  const cx<T>* p = col + phys(g);
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int k = (g + G * b) % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = G * b + r * NB;
      cx<T> x = p[c + c / 8];
      if constexpr (NS > 1) {
        if (r > 0) x = cmul(x, stage_tw<T, NS, R, INV>(twst, k, r));
      }
      v[b][r] = x;
    }
    dftr<T, R, INV>(v[b]);
  }
}

template <typename T, int LEN, int G, int NS, int R, int PB>
__device__ __forceinline__ void stage_to_lds_off(const cx<T> (&v)[PB][R], cx<T>* col, int g) {
#pragma unroll
  for (int b = 0; b < PB; ++b) {
    const int j = g + G * b;
    const int base = (j / NS) * NS * R + (j % NS);
    cx<T>* p = col + phys(base);
#pragma unroll
    for (int r = 0; r < R; ++r) p[r * NS + (r * NS) / 8] = v[b][r];
  }
}

template <typename T, int LEN, int G, int NS, bool INV, bool WAVE_ONLY = false>
__device__ __forceinline__ void middle_stages_off(cx<T>* cola, cx<T>* colb, int g, const cx<T>* __restrict__ twst) {
  constexpr int R = stage_radix<LEN, NS>();
  if constexpr (NS * R < LEN) {
    constexpr int PB = (LEN / R) / G;
    cx<T> va[PB][R], vb[PB][R];
    stage_from_lds_off<T, LEN, G, NS, R, PB, INV>(va, cola, g, twst);
    stage_from_lds_off<T, LEN, G, NS, R, PB, INV>(vb, colb, g, twst);
    stage_sync<WAVE_ONLY>();
    stage_to_lds_off<T, LEN, G, NS, R, PB>(va, cola, g);
    stage_to_lds_off<T, LEN, G, NS, R, PB>(vb, colb, g);
    stage_sync<WAVE_ONLY>();
    middle_stages_off<T, LEN, G, NS * R, INV, WAVE_ONLY>(cola, colb, g, twst);
  }
}

template <typename T, int LEN, int G, int NS, bool INV>
__device__ __forceinline__ void middle_stages1_off(cx<T>* col, int g, const cx<T>* __restrict__ twst) {
  constexpr int R = stage_radix<LEN, NS>();
  if constexpr (NS * R < LEN) {
    constexpr int PB = (LEN / R) / G;
    cx<T> v[PB][R];
    stage_from_lds_off<T, LEN, G, NS, R, PB, INV>(v, col, g, twst);
    __syncthreads();
    stage_to_lds_off<T, LEN, G, NS, R, PB>(v, col, g);
    __syncthreads();
    middle_stages1_off<T, LEN, G, NS * R, INV>(col, g, twst);
  }
}

// Element o of a series as a 32-bit byte offset from a uniform base (loads and stores
// then take the scalar-base form instead of 64-bit vector addresses).
template <typename T>
__device__ __forceinline__ cx<T>& at32(cx<T>* base, unsigned o) {
  return *reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(base) + o * (unsigned)sizeof(cx<T>));
}
template <typename T>
__device__ __forceinline__ const cx<T>& at32(const cx<T>* base, unsigned o) {
  return *reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(base) + o * (unsigned)sizeof(cx<T>));
}

// The intermediate between the two passes holds a template's two series interleaved:
// value (k2, j1) of series s at 2 (k2 P + j1) + s, so that the pair (a, b) of one
// position is one 16-byte access in FP32 and eight adjacent columns fill a 128-byte line.
// It is stored non-temporally: a launch's intermediate (GBs) is read back only after the
// whole launch, so caching it only leaves dirty lines whose write-back competes with the
// second pass's reads (0.71 against 0.68 us per template for that pass).
typedef float f4v_t __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ void store_pair(cx<T>* base, unsigned o, cx<T> a, cx<T> b) {
  if constexpr (sizeof(T) == 4) {
    __builtin_nontemporal_store(f4v_t{a.re, a.im, b.re, b.im},
                                reinterpret_cast<f4v_t*>(reinterpret_cast<char*>(base) + o * 16u));
  } else {
    at32(base, 2 * o) = a;
    at32(base, 2 * o + 1) = b;
  }
}

// Middle stages (stride NS up to, not including, the last stage) for two series.
template <typename T, int LEN, int G, int NS, bool INV, bool WAVE_ONLY = false>
__device__ __forceinline__ void middle_stages(cx<T>* cola, cx<T>* colb, int g, const cx<T>* __restrict__ twst) {
  constexpr int R = stage_radix<LEN, NS>();
  if constexpr (NS * R < LEN) {
    constexpr int PB = (LEN / R) / G;
    cx<T> va[PB][R], vb[PB][R];
    stage_from_lds<T, LEN, G, NS, R, PB, INV>(va, cola, g, twst);
    stage_from_lds<T, LEN, G, NS, R, PB, INV>(vb, colb, g, twst);
    stage_sync<WAVE_ONLY>();
    stage_to_lds<T, LEN, G, NS, R, PB>(va, cola, g);
    stage_to_lds<T, LEN, G, NS, R, PB>(vb, colb, g);
    stage_sync<WAVE_ONLY>();
    middle_stages<T, LEN, G, NS * R, INV, WAVE_ONLY>(cola, colb, g, twst);
  }
}

template <int LEN, int NS>
__host__ __device__ constexpr int last_ns() {
  if constexpr (NS * stage_radix<LEN, NS>() >= LEN) return NS;
  else return last_ns<LEN, NS * stage_radix<LEN, NS>()>();
}

// Forward 8-point DFT of x[0 .. RNZ-1] with x[RNZ ..] = 0 (3 <= RNZ <= 7), in place:
// X[k] = E[k mod 4] + W8^k O[k mod 4], E and O the 4-point DFTs of the even and odd inputs,
// whose zero inputs are left out.  With at most four nonzero inputs the first radix-2
// layer of each 4-point DFT is a copy.
template <typename T, int NZ>
__device__ __forceinline__ void dft4_nz(cx<T> a, cx<T> b, cx<T> c, cx<T> d, cx<T>& y0, cx<T>& y1, cx<T>& y2,
                                        cx<T>& y3) {
  // inputs a, b, c, d with only the first NZ nonzero; y_k = sum x_n (-i)^(nk)
  if constexpr (NZ == 1) {
    y0 = y1 = y2 = y3 = a;
    return;
  }
  cx<T> s0, d0, s1, d1;
  if constexpr (NZ >= 3) {
    s0 = a + c;
    d0 = a - c;
  } else {
    s0 = d0 = a;
  }
  if constexpr (NZ >= 4) {
    s1 = b + d;
    d1 = b - d;
  } else {
    s1 = d1 = b;
  }
  y0 = s0 + s1;
  y2 = s0 - s1;
  y1 = mk<T>(d0.re + d1.im, d0.im - d1.re);
  y3 = mk<T>(d0.re - d1.im, d0.im + d1.re);
}

template <typename T, int RNZ>
__device__ __forceinline__ void dft8_pruned(cx<T>* v) {
  static_assert(RNZ >= 3 && RNZ <= 7, "pruned first stage");
  const T h = (T)0.70710678118654752440084436210485;
  const cx<T> z = mk<T>(0, 0);
  // even inputs x0 x2 x4 x6: (RNZ + 1) / 2 nonzero; odd inputs x1 x3 x5 x7: RNZ / 2
  cx<T> e0, e1, e2, e3, o0, o1, o2, o3;
  dft4_nz<T, (RNZ + 1) / 2>(v[0], v[2], RNZ > 4 ? v[4] : z, RNZ > 6 ? v[6] : z, e0, e1, e2, e3);
  dft4_nz<T, RNZ / 2>(v[1], v[3], RNZ > 5 ? v[5] : z, z, o0, o1, o2, o3);
  // W8^k O[k]: k = 1: h (1 - i), k = 2: -i, k = 3: h (-1 - i)
  const cx<T> w1 = mk<T>(h * (o1.re + o1.im), h * (o1.im - o1.re));
  const cx<T> w2 = mul_mi<T, false>(o2);
  const cx<T> w3 = mk<T>(h * (o3.im - o3.re), -h * (o3.re + o3.im));
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + w1;
  v[5] = e1 - w1;
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = e3 + w3;
  v[7] = e3 - w3;
}

// First stage of pass A for both series: y[j1 + P j2], j2 = j + NB1 r (zero for
// j1 + P j2 >= n), times the template's chirp exp(-2 pi i (c2 jj + c1) jj) at sample jj
// (the spindown phase, plus a lattice grid's frequency shift) whose phase is evaluated
// in FP64 and reduced to [0, 1) cycles, then a radix-R1 DFT in registers.
// All loads are issued before any chirp is computed so that they overlap.  RNZ < R1
// states that inputs r >= RNZ are zero for every column (n <= RNZ L / 8, L the transform
// length), so they are neither loaded nor transformed.
template <typename T, int Q, int G, int R1, int NB1, int PB1, int RNZ = R1>
__device__ __forceinline__ void chirped_first_stage(cx<T> (&va)[PB1][R1], cx<T> (&vb)[PB1][R1],
                                                    const cx<T>* __restrict__ za, const cx<T>* __restrict__ zb,
                                                    int j1, int g, int P, int n, double c2, double c1) {
#pragma unroll
  for (int b = 0; b < PB1; ++b) {
    const unsigned j = (unsigned)(g + G * b);
#pragma unroll
    for (int r = 0; r < RNZ; ++r) {
      const unsigned jj = (unsigned)j1 + (unsigned)P * (j + (unsigned)(NB1 * r));
      va[b][r] = mk<T>(0, 0);
      vb[b][r] = mk<T>(0, 0);
      if (jj < (unsigned)n) {
        va[b][r] = at32(za, jj);
        vb[b][r] = at32(zb, jj);
      }
    }
#pragma unroll
    for (int r = 0; r < RNZ; ++r) {
      const unsigned jj = (unsigned)j1 + (unsigned)P * (j + (unsigned)(NB1 * r));
      if (jj < (unsigned)n) {
        const double x = (double)jj;
        double cyc = fma(c2, x, c1) * x;
        cyc -= floor(cyc);
        T s, co;
        if constexpr (sizeof(T) == 8) {
          sincospi(2.0 * cyc, &s, &co);
        } else {
          // the hardware sine and cosine take their argument in cycles
          const float cf = (float)cyc;
          s = __builtin_amdgcn_sinf(cf);
          co = __builtin_amdgcn_cosf(cf);
        }
        const cx<T> w = mk<T>(co, -s);
        va[b][r] = cmul(va[b][r], w);
        vb[b][r] = cmul(vb[b][r], w);
      }
    }
    if constexpr (RNZ < R1) {
      static_assert(R1 == 8, "pruning is for radix-8 first stages");
      dft8_pruned<T, RNZ>(va[b]);
      dft8_pruned<T, RNZ>(vb[b]);
    } else {
      dftr<T, R1, false>(va[b]);
      dftr<T, R1, false>(vb[b]);
    }
  }
}

// ---------------------------------------------------------------- pass A
// Workgroup: TW adjacent columns j1 of one template; thread (c = t % TW, g = t / TW).
// The two series share the chirp; they pass through one LDS tile one after the
// other, the second series' first-stage outputs waiting in registers.
template <typename T, int Q, int RNZ = stage_radix<Q, 1>()>
__global__ void __launch_bounds__((tmpl_nt_a<T, Q>())) k_tmpl_a(TmplArgs ta, const cx<T>* __restrict__ zt,
                                                           cx<T>* __restrict__ tbuf,
                                                           const cx<T>* __restrict__ twst,
                                                           const cx<T>* __restrict__ twlo,
                                                           const cx<T>* __restrict__ twhi) {
  constexpr int G = groups_per_col<Q>();
  constexpr int TW = tw_a<T, Q>();
  constexpr int ST = col_stride<Q>(want_a<TW>());
  constexpr int R1 = stage_radix<Q, 1>();
  constexpr int NB1 = Q / R1, PB1 = NB1 / G;
  static_assert(PB1 >= 1 && NB1 % G == 0, "first stage must give each thread whole butterflies");
  static_assert(R1 < Q, "at least two stages");
  __shared__ cx<T> lds[TW * ST];
  int tile, item;
  xcd_tile_item(ta.P / TW, tile, item);
  const int c = threadIdx.x % TW, g = threadIdx.x / TW;
  const int t = ta.t0 + item;
  const int skyl = t / ta.nfdot, sidx = t % ta.nfdot;
  double c2, c1;
  template_chirp(ta, skyl, sidx, c2, c1);
  const cx<T>* za = zt + (long)(2 * skyl) * ta.ldzt;
  const cx<T>* zb = za + ta.ldzt;
  const int j1 = tile * TW + c;
  cx<T>* col = lds + c * ST;
  // first stage: y[j1 + P j2] with the spindown chirp, radix-R1 butterflies in registers
  cx<T> va[PB1][R1], vb[PB1][R1];
  chirped_first_stage<T, Q, G, R1, NB1, PB1, RNZ>(va, vb, za, zb, j1, g, ta.P, ta.n, c2, c1);
  // twiddles W^(j1 k2) of the last-stage outputs k2 = j + NSL r: W^(j1 j) times powers of W^(j1 NSL)
  constexpr int NSL = last_ns<Q, 1>();
  constexpr int RL = stage_radix<Q, NSL>();
  constexpr int PBL = (Q / RL) / G;
  cx<T> tw[PBL][RL];
  {
    const cx<T> step = twiddle_L<T, false>(twlo, twhi, j1 * NSL);
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
      cx<T> w = twiddle_L<T, false>(twlo, twhi, j1 * (g + G * b));
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        tw[b][r] = w;
        if (r + 1 < RL) w = cmul(w, step);
      }
    }
  }
  // series a's outputs wait in registers so that both series leave as (a, b) pairs
  cx<T> ka[PBL][RL];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s == 1) __syncthreads();  // series a's last stage has read the tile
    stage_to_lds_off<T, Q, G, 1, R1, PB1>(s == 0 ? va : vb, col, g);
    __syncthreads();
    middle_stages1_off<T, Q, G, R1, false>(col, g, twst);
    cx<T> v[PBL][RL];
    stage_from_lds_off<T, Q, G, NSL, RL, PBL, false>(v, col, g, twst);
    cx<T>* out = tbuf + (long)(2 * item) * ta.L;
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
      const int j = g + G * b;
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const unsigned o = (unsigned)(j + NSL * r) * (unsigned)ta.P + (unsigned)j1;
        if (s == 0) ka[b][r] = cmul(v[b][r], tw[b][r]);
        else store_pair(out, o, ka[b][r], cmul(v[b][r], tw[b][r]));
      }
    }
  }
}

// Pass A, paired variant: both series in LDS at once (twice the tile, half the
// barriers).  The same operations as k_tmpl_a (the compiler may contract
// multiply-adds differently, so results can differ in the last bit).
template <typename T, int Q, int RNZ = stage_radix<Q, 1>()>
__global__ void __launch_bounds__((tmpl_nt_a<T, Q>())) k_tmpl_a_pair(TmplArgs ta, const cx<T>* __restrict__ zt,
                                                                cx<T>* __restrict__ tbuf,
                                                                const cx<T>* __restrict__ twst,
                                                                const cx<T>* __restrict__ twlo,
                                                                const cx<T>* __restrict__ twhi) {
  constexpr int G = groups_per_col<Q>();
  constexpr int TW = tw_a<T, Q>();
  constexpr int ST = col_stride<Q>(want_a<TW>());
  constexpr int R1 = stage_radix<Q, 1>();
  constexpr int NB1 = Q / R1, PB1 = NB1 / G;
  static_assert(PB1 >= 1 && NB1 % G == 0, "first stage must give each thread whole butterflies");
  static_assert(R1 < Q, "at least two stages");
  __shared__ cx<T> lds[2 * TW * ST];
  int tile, item;
  xcd_tile_item(ta.P / TW, tile, item);
  const int c = threadIdx.x % TW, g = threadIdx.x / TW;
  const int t = ta.t0 + item;
  const int skyl = t / ta.nfdot, sidx = t % ta.nfdot;
  double c2, c1;
  template_chirp(ta, skyl, sidx, c2, c1);
  const cx<T>* za = zt + (long)(2 * skyl) * ta.ldzt;
  const cx<T>* zb = za + ta.ldzt;
  const int j1 = tile * TW + c;
  cx<T>* cola = lds + c * ST;
  cx<T>* colb = lds + (TW + c) * ST;
  {
    cx<T> va[PB1][R1], vb[PB1][R1];
    chirped_first_stage<T, Q, G, R1, NB1, PB1, RNZ>(va, vb, za, zb, j1, g, ta.P, ta.n, c2, c1);
    stage_to_lds_off<T, Q, G, 1, R1, PB1>(va, cola, g);
    stage_to_lds_off<T, Q, G, 1, R1, PB1>(vb, colb, g);
    __syncthreads();
  }
  middle_stages_off<T, Q, G, R1, false>(cola, colb, g, twst);
  constexpr int NSL = last_ns<Q, 1>();
  constexpr int RL = stage_radix<Q, NSL>();
  constexpr int PBL = (Q / RL) / G;
  cx<T> va[PBL][RL], vb[PBL][RL];
  stage_from_lds_off<T, Q, G, NSL, RL, PBL, false>(va, cola, g, twst);
  stage_from_lds_off<T, Q, G, NSL, RL, PBL, false>(vb, colb, g, twst);
  cx<T>* out = tbuf + (long)(2 * item) * ta.L;
  const cx<T> step = twiddle_L<T, false>(twlo, twhi, j1 * NSL);
#pragma unroll
  for (int b = 0; b < PBL; ++b) {
    const int j = g + G * b;
    cx<T> w = twiddle_L<T, false>(twlo, twhi, j1 * j);
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const unsigned o = (unsigned)(j + NSL * r) * (unsigned)ta.P + (unsigned)j1;
      store_pair(out, o, cmul(va[b][r], w), cmul(vb[b][r], w));
      if (r + 1 < RL) w = cmul(w, step);
    }
  }
}

// 2F = cfa |Fa|^2 + cfb |Fb|^2 + cfab Re(Fa Fb*) with every rounding spelled out, so that
// the threshold, the spectrum store and the patch capture see bitwise the same value.
__device__ __forceinline__ float two_f_value(cx<float> fa, cx<float> fb, float cfa, float cfb, float cfab) {
  const float na = __fmaf_rn(fa.re, fa.re, __fmul_rn(fa.im, fa.im));
  const float nb = __fmaf_rn(fb.re, fb.re, __fmul_rn(fb.im, fb.im));
  const float xr = __fmaf_rn(fa.re, fb.re, __fmul_rn(fa.im, fb.im));
  return __fmaf_rn(cfa, na, __fmaf_rn(cfb, nb, __fmul_rn(cfab, xr)));
}
// The same value when cfab = 0 (the simplified form): fma(cfb, nb, 0 * xr) rounds as cfb * nb.
__device__ __forceinline__ float two_f_value_nc(cx<float> fa, cx<float> fb, float cfa, float cfb) {
  const float na = __fmaf_rn(fa.re, fa.re, __fmul_rn(fa.im, fa.im));
  const float nb = __fmaf_rn(fb.re, fb.re, __fmul_rn(fb.im, fb.im));
  return __fmaf_rn(cfa, na, __fmul_rn(cfb, nb));
}
__device__ __forceinline__ double two_f_value(cx<double> fa, cx<double> fb, double cfa, double cfb, double cfab) {
  const double na = __fma_rn(fa.re, fa.re, __dmul_rn(fa.im, fa.im));
  const double nb = __fma_rn(fb.re, fb.re, __dmul_rn(fb.im, fb.im));
  const double xr = __fma_rn(fa.re, fb.re, __dmul_rn(fa.im, fb.im));
  return __fma_rn(cfa, na, __fma_rn(cfb, nb, __dmul_rn(cfab, xr)));
}

// ---------------------------------------------------------------- pass B
// Workgroup: TW adjacent rows k2 of one template; thread (c = t / G, g = t % G).
template <typename T, int P, int MODE>
__global__ void __launch_bounds__((tmpl_nt_b<T, P>())) k_tmpl_b(TmplArgs ta, const SkyParams* __restrict__ sp,
                                                           const cx<T>* __restrict__ tbuf, OutArgs oa,
                                                           const cx<T>* __restrict__ twst) {
  constexpr int NTB = tmpl_nt_b<T, P>();
  constexpr int G = groups_per_col<P>();
  constexpr int TW = tw_b<T, P>();
  constexpr int ST = col_stride<P>(16);
  constexpr int R1 = stage_radix<P, 1>();
  constexpr int NB1 = P / R1, PB1 = NB1 / G;
  static_assert(TW * G == NTB, "one butterfly group per thread");
  __shared__ cx<T> lds[2 * TW * ST];
  __shared__ unsigned long long sbase;
  int tile, item;
  xcd_tile_item(ta.Q / TW, tile, item);
  const int c = threadIdx.x / G, g = threadIdx.x % G;
  const int t = ta.t0 + item;
  const int skyl = t / ta.nfdot, sidx = t % ta.nfdot;
  const int k2 = tile * TW + c;
  const cx<T>* in = tbuf + (long)(2 * item) * ta.L + 2 * (long)k2 * ta.P;
  cx<T>* cola = lds + c * ST;
  cx<T>* colb = lds + (TW + c) * ST;
  {
    cx<T> va[PB1][R1], vb[PB1][R1];
#pragma unroll
    for (int b = 0; b < PB1; ++b) {
      const int j = g + G * b;
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        va[b][r] = in[2 * (j + NB1 * r)];
        vb[b][r] = in[2 * (j + NB1 * r) + 1];
      }
      dftr<T, R1, false>(va[b]);
      dftr<T, R1, false>(vb[b]);
    }
    stage_to_lds<T, P, G, 1, R1, PB1>(va, cola, g);
    stage_to_lds<T, P, G, 1, R1, PB1>(vb, colb, g);
    stage_sync<rows_in_wave<P>()>();
  }
  middle_stages<T, P, G, R1, false, rows_in_wave<P>()>(cola, colb, g, twst);
  constexpr int NSL = last_ns<P, 1>();
  constexpr int RL = stage_radix<P, NSL>();
  constexpr int PBL = (P / RL) / G;
  constexpr int NOUT = PBL * RL;
  static_assert(NOUT <= 32, "output mask");
  cx<T> va[PBL][RL], vb[PBL][RL];
  stage_from_lds<T, P, G, NSL, RL, PBL, false>(va, cola, g, twst);
  stage_from_lds<T, P, G, NSL, RL, PBL, false>(vb, colb, g, twst);
  if constexpr (MODE == 3) {
    // the transform itself, for an epilogue of its own: oa.spectrum as [item][k][a|b]
    cx<T>* xs = (cx<T>*)oa.spectrum + (long)(2 * item) * ta.L;
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = ta.Q * (g + G * b + NSL * r) + k2;
        xs[2 * k] = va[b][r];
        xs[2 * k + 1] = vb[b][r];
      }
    }
    return;
  }
  const SkyParams& pr = sp[skyl];
  const T cfa = (T)pr.cfa, cfb = (T)pr.cfb, cfab = (T)pr.cfab;
  if constexpr (MODE == 2) {
    // the launch's 2F rows for the patch capture that follows (template-major, FP32)
    float* out = (float*)oa.spectrum + (long)item * (long)(oa.k_max - oa.k_min);
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int klo = ta.Q * (G * b + NSL * r) + k2;
        if (klo < oa.k_max && klo + ta.Q * (G - 1) >= oa.k_min) {
          const int k = ta.Q * (g + G * b + NSL * r) + k2;
          if (k >= oa.k_min && k < oa.k_max) {
            const cx<T> fa = va[b][r], fb = vb[b][r];
            out[k - oa.k_min] = (float)two_f_value(fa, fb, cfa, cfb, cfab);
          }
        }
      }
    }
  }
  if constexpr (MODE == 1) {
    T* out = (T*)oa.spectrum + ((long)(ta.sky0 + skyl) * ta.nfdot + sidx) * (long)(oa.k_max - oa.k_min);
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = ta.Q * (g + G * b + NSL * r) + k2;
        if (k >= oa.k_min && k < oa.k_max) {
          const cx<T> fa = va[b][r], fb = vb[b][r];
          out[k - oa.k_min] = two_f_value(fa, fb, cfa, cfb, cfab);
        }
      }
    }
  } else {  // MODE 0 and 2: threshold and compaction
    uint32_t mask = 0;
    T val[NOUT];
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        val[b * RL + r] = (T)0;
        // bins of this output group: k = Q (G b + NSL r + g') + k2 over the G lanes g'
        const int klo = ta.Q * (G * b + NSL * r) + k2;
        if (klo < oa.k_max && klo + ta.Q * (G - 1) >= oa.k_min) {
          const int k = ta.Q * (g + G * b + NSL * r) + k2;
          const cx<T> fa = va[b][r], fb = vb[b][r];
          const T v = two_f_value(fa, fb, cfa, cfb, cfab);
          val[b * RL + r] = v;
          if (k >= oa.k_min && k < oa.k_max && v > (T)oa.threshold) mask |= 1u << (b * RL + r);
        }
      }
    }
    int total;
    const int off = block_exclusive_scan_n<NTB>(__popc(mask), &total);
    if (total == 0) return;
    if (threadIdx.x == 0) sbase = atomicAdd(oa.count, (unsigned long long)total);
    __syncthreads();
    const int search = oa.search_next[0] - 1;
    unsigned long long slot = sbase + (unsigned long long)off;
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
      if (mask & (1u << i)) {
        if (slot < (unsigned long long)oa.capacity) {
          const int b = i / RL, r = i % RL;
          CandEntry ce;
          ce.search = search;
          ce.segment = oa.segment;
          ce.sky = ta.sky0 + skyl;
          ce.fdot_idx = sidx;
          ce.bin = ta.Q * (g + G * b + NSL * r) + k2;
          ce.pad = 0;
          ce.twoF = (double)val[i];
          oa.cand[slot] = ce;
        }
        ++slot;
      }
    }
  }
}

// ------------------------------------------------ interbinned 2F from stored transforms (FP64)
// The tiled second pass (mode 3) has stored each template's transform of L points,
// xs = [item][k][a|b].  Bin 2k of the nfft grid is X_k and bin 2k + 1 is
// c (X_k - X_{k+1 mod L}), for both series; 2F, threshold and compaction as in the
// tiled pass (one atomic per workgroup).  Grid: (coarse-bin blocks, templates of the
// launch); thread = one coarse bin k in [kc0, kc0 + nkc).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_interbin_2f(TmplArgs ta, const SkyParams* __restrict__ sp,
                                                     const cx<T>* __restrict__ xs, OutArgs oa, double c, int kc0,
                                                     int nkc) {
  __shared__ unsigned long long sbase;
  const int item = blockIdx.y;
  const int t = ta.t0 + item;
  const int skyl = t / ta.nfdot, sidx = t % ta.nfdot;
  const int kc = kc0 + (int)blockIdx.x * 256 + (int)threadIdx.x;
  const SkyParams& pr = sp[skyl];
  const T cfa = (T)pr.cfa, cfb = (T)pr.cfb, cfab = (T)pr.cfab;
  T v[2] = {(T)0, (T)0};
  bool in[2] = {false, false};
  if (kc < kc0 + nkc) {
    const cx<T>* x = xs + (long)(2 * item) * ta.L;
    const int kn = kc + 1 == ta.L ? 0 : kc + 1;
    const cx<T> a0 = x[2 * kc], b0 = x[2 * kc + 1], a1 = x[2 * kn], b1 = x[2 * kn + 1];
    const T w = (T)c;
    const cx<T> da = a0 - a1, db = b0 - b1;
    v[0] = two_f_value(a0, b0, cfa, cfb, cfab);
    v[1] = two_f_value(mk<T>(w * da.re, w * da.im), mk<T>(w * db.re, w * db.im), cfa, cfb, cfab);
#pragma unroll
    for (int e = 0; e < 2; ++e) in[e] = 2 * kc + e >= oa.k_min && 2 * kc + e < oa.k_max;
  }
  if constexpr (MODE == 1) {
    T* out = (T*)oa.spectrum + ((long)(ta.sky0 + skyl) * ta.nfdot + sidx) * (long)(oa.k_max - oa.k_min);
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (in[e]) out[2 * kc + e - oa.k_min] = v[e];
    return;
  }
  if constexpr (MODE == 2) {
    float* out = (float*)oa.spectrum + (long)item * (long)(oa.k_max - oa.k_min);
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (in[e]) out[2 * kc + e - oa.k_min] = (float)v[e];
  }
  uint32_t mask = 0;
#pragma unroll
  for (int e = 0; e < 2; ++e)
    if (in[e] && v[e] > (T)oa.threshold) mask |= 1u << e;
  int total;
  const int off = block_exclusive_scan_n<256>(__popc(mask), &total);
  if (total == 0) return;
  if (threadIdx.x == 0) sbase = atomicAdd(oa.count, (unsigned long long)total);
  __syncthreads();
  const int search = oa.search_next[0] - 1;
  unsigned long long slot = sbase + (unsigned long long)off;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    if (mask & (1u << e)) {
      if (slot < (unsigned long long)oa.capacity) {
        CandEntry ce;
        ce.search = search;
        ce.segment = oa.segment;
        ce.sky = ta.sky0 + skyl;
        ce.fdot_idx = sidx;
        ce.bin = 2 * kc + e;
        ce.pad = 0;
        ce.twoF = (double)v[e];
        oa.cand[slot] = ce;
      }
      ++slot;
    }
  }
}

// ---------------------------------------------------------------- pass B, streaming (FP32, P <= 512)
// Each wavefront owns RPW = 64 / G whole rows and walks NR row units of one template.  The eight paired (a, b) loads of the next unit are issued before the current
// unit is transformed, so HBM reads overlap the butterflies; twiddles of the stages
// after the first stay in registers for the whole walk; all LDS exchanges are local to
// the wavefront; candidates are compacted with ballots and one atomic per wavefront
// and unit that has any.  When the searched bins are exactly [0, nfft/2) (HALF), the
// last stage computes only the outputs k1 < P/2 and no bin needs a range check.

// Twiddles of the stage at stride NS and of all later stages, for butterflies j = g + G b.
template <typename T, int LEN, int G, int NS, bool MORE = (NS < LEN)>
struct StageTw {
  static constexpr int R = stage_radix<LEN, NS>();
  static constexpr int PB = (LEN / R) / G;
  cx<T> w[PB][R - 1];
  StageTw<T, LEN, G, NS * R> next;
  __device__ __forceinline__ void load(const cx<T>* __restrict__ twst, int g) {
#pragma unroll
    for (int b = 0; b < PB; ++b)
#pragma unroll
      for (int r = 1; r < R; ++r) w[b][r - 1] = stage_tw<T, NS, R, false>(twst, (g + G * b) % NS, r);
    next.load(twst, g);
  }
};
template <typename T, int LEN, int G, int NS>
struct StageTw<T, LEN, G, NS, false> {
  __device__ __forceinline__ void load(const cx<T>* __restrict__, int) {}
};

// The first R/2 outputs of a forward R-point DFT (v[0 .. R/2 - 1]; the rest is garbage).
// Even outputs are the R/2-point DFT of x[n] + x[n + R/2], odd ones that of
// (x[n] - x[n + R/2]) W_R^n, of which only the first halves are formed.
template <typename T, int R>
__device__ __forceinline__ void dft_first_half(cx<T>* v) {
  if constexpr (R == 2) {
    v[0] = v[0] + v[1];
  } else if constexpr (R == 4) {
    const cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
    const cx<T> s13 = v[1] + v[3], d13 = mul_mi<T, false>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[1] = d02 + d13;
  } else {
    const T h = (T)0.70710678118654752440084436210485;
    const cx<T> a0 = v[0] + v[4], a1 = v[1] + v[5], a2 = v[2] + v[6], a3 = v[3] + v[7];
    const cx<T> d0 = v[0] - v[4], e1 = v[1] - v[5], e2 = v[2] - v[6], e3 = v[3] - v[7];
    const cx<T> d1 = mk<T>(h * (e1.re + e1.im), h * (e1.im - e1.re));
    const cx<T> d2 = mul_mi<T, false>(e2);
    const cx<T> d3 = mk<T>(h * (e3.im - e3.re), -h * (e3.re + e3.im));
    v[0] = (a0 + a2) + (a1 + a3);
    v[2] = (a0 - a2) + mul_mi<T, false>(a1 - a3);
    v[1] = (d0 + d2) + (d1 + d3);
    v[3] = (d0 - d2) + mul_mi<T, false>(d1 - d3);
  }
}

// Stage loads and stores addressed as one base plus compile-time offsets: for the strides
// used here phys(a + c) = phys(a) + c + c/8 (c a multiple of 8, or a % 8 + c < 8).
template <typename T, int LEN, int G, int NS, int R, int PB, bool HALFOUT>
__device__ __forceinline__ void stage_from_lds_reg(cx<T> (&v)[PB][R], const cx<T>* col, int g,
                                                   const cx<T> (&w)[PB][R - 1]) {
  constexpr int NB = LEN / R;
  static_assert(NB % 8 == 0, "constant offsets need NB a multiple of 8");
  const cx<T>* p = col + phys(g);
#pragma unroll
  for (int b = 0; b < PB; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = G * b + r * NB;  // G * b is a multiple of 8 when PB > 1
      cx<T> x = p[c + c / 8];
      if (r > 0) x = cmul(x, w[b][r - 1]);
      v[b][r] = x;
    }
    if constexpr (HALFOUT) dft_first_half<T, R>(v[b]);
    else dftr<T, R, false>(v[b]);
  }
}

// WAVE_ONLY: the rows belong to single wavefronts (otherwise a workgroup barrier orders
// the stages of rows that span wavefronts).
template <typename T, int LEN, int G, int NS, bool WAVE_ONLY = true>
__device__ __forceinline__ void middle_stages_reg(cx<T>* cola, cx<T>* colb, int g, const StageTw<T, LEN, G, NS>& tw) {
  constexpr int R = stage_radix<LEN, NS>();
  if constexpr (NS * R < LEN) {
    constexpr int PB = (LEN / R) / G;
    cx<T> va[PB][R], vb[PB][R];
    stage_from_lds_reg<T, LEN, G, NS, R, PB, false>(va, cola, g, tw.w);
    stage_from_lds_reg<T, LEN, G, NS, R, PB, false>(vb, colb, g, tw.w);
    stage_sync<WAVE_ONLY>();
    stage_to_lds_off<T, LEN, G, NS, R, PB>(va, cola, g);
    stage_to_lds_off<T, LEN, G, NS, R, PB>(vb, colb, g);
    stage_sync<WAVE_ONLY>();
    middle_stages_reg<T, LEN, G, NS * R, WAVE_ONLY>(cola, colb, g, tw.next);
  }
}

template <typename T, int LEN, int G, int NS>
__device__ __forceinline__ const auto& last_stage_tw(const StageTw<T, LEN, G, NS>& tw) {
  if constexpr (NS * stage_radix<LEN, NS>() >= LEN) return tw;
  else return last_stage_tw<T, LEN, G, NS * stage_radix<LEN, NS>()>(tw.next);
}

// A value of the intermediate, read once: a non-temporal load (the row is not kept in
// the caches for reuse).
__device__ __forceinline__ void load_stream(const cx<float>* p, cx<float>& a, cx<float>& b) {
  const f4v_t v = __builtin_nontemporal_load(reinterpret_cast<const f4v_t*>(p));
  a = mk<float>(v.x, v.y);
  b = mk<float>(v.z, v.w);
}
__device__ __forceinline__ void load_stream(const cx<double>* p, cx<double>& a, cx<double>& b) {
  a = p[0];
  b = p[1];
}

// Candidates a wavefront stages in LDS before it reserves their slots with one atomic.
constexpr int STAGE_CAP = 32;

// Candidate staging of one wavefront in the streaming second passes: crossings are
// compacted with ballots into the wavefront's STAGE_CAP-entry LDS area, and one atomic
// reserves the slots of a whole area (a burst larger than the area goes straight out).
struct WaveStage {
  int* item;
  int* bin;
  float* val;
  int n = 0;

  template <typename T>
  __device__ __forceinline__ static void emit(const OutArgs& oa, const TmplArgs& ta, int search,
                                              unsigned long long slot, int it, int b, T v) {
    if (slot < (unsigned long long)oa.capacity) {
      const int t = ta.t0 + it;
      const int skyl = t / ta.nfdot;
      CandEntry ce;
      ce.search = search;
      ce.segment = oa.segment;
      ce.sky = ta.sky0 + skyl;
      ce.fdot_idx = t - skyl * ta.nfdot;
      ce.bin = b;
      ce.pad = 0;
      ce.twoF = (double)v;
      oa.cand[slot] = ce;
    }
  }

  // `count` slots for the whole wavefront (the same base in every lane)
  __device__ __forceinline__ static unsigned long long reserve(const OutArgs& oa, int lane, int count) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(oa.count, (unsigned long long)count);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)base);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(base >> 32));
    return ((unsigned long long)hi << 32) | lo;
  }

  __device__ __forceinline__ void flush(const OutArgs& oa, const TmplArgs& ta, int search, int lane) {
    if (n == 0) return;
    stage_sync<true>();
    const unsigned long long base = reserve(oa, lane, n);
    if (lane < n) emit(oa, ta, search, base + lane, item[lane], bin[lane], val[lane]);
    stage_sync<true>();
    n = 0;
  }

  // Crossings of this lane: bit q of `mask` for value v[q] of bin bin_of(q), template it.
  // TWO_PASS counts the ballots first and places them in a second round, keeping no
  // per-value offsets (fewer registers for long value lists).
  template <bool TWO_PASS, int NV, typename T, typename BinOf>
  __device__ __forceinline__ void add(const OutArgs& oa, const TmplArgs& ta, int search, int lane, uint32_t mask,
                                      const T (&v)[NV], int it, BinOf bin_of) {
    if (!__ballot(mask != 0)) return;
    auto rank = [&](unsigned long long bi) {
      return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(bi >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bi, 0u));
    };
    int total = 0;
    int off[TWO_PASS ? 1 : NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const unsigned long long bi = __ballot((mask >> q) & 1u);
      if constexpr (!TWO_PASS) off[q] = total + rank(bi);
      total += __popcll(bi);
    }
    if (n + total > STAGE_CAP) flush(oa, ta, search, lane);
    const bool direct = total > STAGE_CAP;
    const unsigned long long base = direct ? reserve(oa, lane, total) : 0ull;
    int run = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      int o;
      if constexpr (TWO_PASS) {
        const unsigned long long bi = __ballot((mask >> q) & 1u);
        o = run + rank(bi);
        run += __popcll(bi);
      } else {
        o = off[q];
      }
      if ((mask >> q) & 1u) {
        if (direct) {
          emit(oa, ta, search, base + (unsigned long long)o, it, bin_of(q), v[q]);
        } else {
          item[n + o] = it;
          bin[n + o] = bin_of(q);
          val[n + o] = (float)v[q];
        }
      }
    }
    if (!direct) n += total;
  }
};

// Columns per block of the 2F rows the streaming second pass stores for the patch capture.
constexpr int CAP_BLOCK = 8;

// Row units per wavefront step: RPW rows of P points.
template <int P>
__host__ __device__ constexpr int stream_rpw() { return 64 / groups_per_col<P>(); }

template <typename T, int P, int MODE, bool HALF>
__global__ void __launch_bounds__(256) k_tmpl_b_stream(TmplArgs ta, int ntmpl, const SkyParams* __restrict__ sp,
                                                       const cx<T>* __restrict__ tbuf, OutArgs oa,
                                                       const cx<T>* __restrict__ twst) {
  constexpr int G = groups_per_col<P>();
  static_assert(G <= 64 && 64 % G == 0, "rows must tile a wavefront");
  constexpr int RPW = stream_rpw<P>();
  constexpr int ST = col_stride<P>(16);
  constexpr int R1 = stage_radix<P, 1>();
  constexpr int NB1 = P / R1, PB1 = NB1 / G;
  static_assert(PB1 >= 1 && NB1 % G == 0, "first stage must give each lane whole butterflies");
  constexpr int NSL = last_ns<P, 1>();
  constexpr int RL = stage_radix<P, NSL>();
  constexpr int PBL = (P / RL) / G;
  constexpr int ROUT = HALF ? RL / 2 : RL;
  constexpr int NOUT = PBL * ROUT;
  static_assert(NOUT <= 32, "output mask");
  __shared__ cx<T> lds[4 * 2 * RPW * ST];
  // per-wavefront candidate staging: (template of the launch, bin, 2F)
  __shared__ int st_item[4][STAGE_CAP];
  __shared__ int st_bin[4][STAGE_CAP];
  __shared__ float st_val[4][STAGE_CAP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int units = ta.Q / RPW;        // row units of one template
  const int total = ntmpl * units;     // row units of the launch
  const int nw = gridDim.x * 4;        // wavefronts of the grid
  const int sub = lane / G, g = lane % G;
  cx<T>* cola = lds + (wave * 2 * RPW + sub) * ST;
  cx<T>* colb = cola + RPW * ST;
  const T thr = (T)oa.threshold;
  const int search = oa.search_next[0] - 1;
  StageTw<T, P, G, R1> tw;
  tw.load(twst, g);
  const auto& twl = last_stage_tw<T, P, G, R1>(tw);
  const int lofs = sub * P + g;

  // unit U of the launch: template U / units, rows (U % units) RPW + sub
  auto load_unit = [&](cx<T> (&ca)[PB1][R1], cx<T> (&cb)[PB1][R1], int U) {
    const int item = U / units, u = U - item * units;
    const cx<T>* p = tbuf + (long)(2 * item) * ta.L + 2 * (long)u * (RPW * P);
#pragma unroll
    for (int b = 0; b < PB1; ++b)
#pragma unroll
      for (int r = 0; r < R1; ++r) load_stream(p + 2 * (lofs + G * b + NB1 * r), ca[b][r], cb[b][r]);
  };

  WaveStage stg{st_item[wave], st_bin[wave], st_val[wave]};

  // Wavefront w takes units w, w + nw, w + 2 nw, ...: the grid is about one resident
  // round of wavefronts, so the rows being read at any time form one contiguous window.
  int U = blockIdx.x * 4 + wave;
  if (U >= total) return;
  cx<T> xa[PB1][R1], xb[PB1][R1];
  load_unit(xa, xb, U);
  for (; U < total; U += nw) {
    const int item = U / units;
    const int u = U - item * units;
    const int t = ta.t0 + item;
    const int skyl = t / ta.nfdot, sidx = t - skyl * ta.nfdot;
    const SkyParams& pr = sp[skyl];
    const T cfa = (T)pr.cfa, cfb = (T)pr.cfb, cfab = (T)pr.cfab;
#pragma unroll
    for (int b = 0; b < PB1; ++b) {
      dftr<T, R1, false>(xa[b]);
      dftr<T, R1, false>(xb[b]);
    }
    stage_sync<true>();  // the previous unit's last stage has read the slab
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xa, cola, g);
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xb, colb, g);
    stage_sync<true>();
    // the next unit's loads go into the registers just freed and overlap the rest
    if (U + nw < total) load_unit(xa, xb, U + nw);
    middle_stages_reg<T, P, G, R1>(cola, colb, g, tw);
    cx<T> fa[PBL][RL], fb[PBL][RL];
    stage_from_lds_reg<T, P, G, NSL, RL, PBL, HALF>(fa, cola, g, twl.w);
    stage_from_lds_reg<T, P, G, NSL, RL, PBL, HALF>(fb, colb, g, twl.w);
    const int k2 = u * RPW + sub;
    if constexpr (MODE == 1) {
      T* out = (T*)oa.spectrum + ((long)(ta.sky0 + skyl) * ta.nfdot + sidx) * (long)(oa.k_max - oa.k_min);
#pragma unroll
      for (int b = 0; b < PBL; ++b)
#pragma unroll
        for (int r = 0; r < ROUT; ++r) {
          const int k = ta.Q * (g + G * b + NSL * r) + k2;
          if (HALF || (k >= oa.k_min && k < oa.k_max))
            out[k - oa.k_min] = two_f_value(fa[b][r], fb[b][r], cfa, cfb, cfab);
        }
    } else {
      // MODE 2 (patch capture) stores the launch's 2F values in blocks of eight columns,
      // [template][k1 / 8][k2][k1 % 8] (RLEN columns: the outputs a row forms): eight lanes
      // store 32 contiguous bytes, the lines filled by the neighbouring rows that other
      // wavefronts form at the same time, and a window's 256 consecutive bins (consecutive
      // k2, one or two k1) lie four to a 128-byte line
      constexpr int RLEN = HALF ? P / 2 : P;
      static_assert(RLEN % CAP_BLOCK == 0, "whole column blocks");
      float* srow = (float*)oa.spectrum + (long)item * ta.Q * RLEN + (long)k2 * CAP_BLOCK;
      uint32_t mask = 0;
      T val[NOUT];
#pragma unroll
      for (int b = 0; b < PBL; ++b)
#pragma unroll
        for (int r = 0; r < ROUT; ++r) {
          const int k1 = g + G * b + NSL * r;
          const int k = ta.Q * k1 + k2;
          const T v = two_f_value(fa[b][r], fb[b][r], cfa, cfb, cfab);
          val[b * ROUT + r] = v;
          const bool inr = HALF || (k >= oa.k_min && k < oa.k_max);
          if (MODE == 2) srow[(long)(k1 / CAP_BLOCK) * ta.Q * CAP_BLOCK + k1 % CAP_BLOCK] = (float)v;
          if (inr && v > thr) mask |= 1u << (b * ROUT + r);
        }
      stg.add<false>(oa, ta, search, lane, mask, val, item,
                     [&](int q) { return ta.Q * (g + G * (q / ROUT) + NSL * (q % ROUT)) + k2; });
    }
  }
  if constexpr (MODE != 1) stg.flush(oa, ta, search, lane);
}

// ---------------------------------------------------------------- pass B, streaming, rows of 1024 points (FP32)
// A row of P = 1024 points has 128 radix-8 butterflies per stage, so it spans two
// wavefronts; a workgroup of NT threads transforms the NT / 128 rows k2 = u NT / 128 + i of
// one template (row unit u) per step and walks the launch's units with the grid as stride,
// so that the rows being read at any time form one contiguous window of HBM.  As in
// k_tmpl_b_stream, the next unit's paired (a, b) loads are issued once the first stage is
// in LDS and overlap the remaining stages, and the later stages' twiddles stay in
// registers; workgroup barriers order the stages.  MODE 0: threshold and candidates
// (staged per wavefront), MODE 1: the 2F spectrum.  With HALF (bins [0, nfft/2)) the
// radix-2 last stage forms only the outputs k1 < P/2.
template <int MODE, bool HALF, int NT>
__global__ void __launch_bounds__(NT) k_tmpl_b_stream2(TmplArgs ta, int ntmpl, const SkyParams* __restrict__ sp,
                                                        const cx<float>* __restrict__ tbuf, OutArgs oa,
                                                        const cx<float>* __restrict__ twst) {
  using T = float;
  constexpr int P = 1024;
  constexpr int G = groups_per_col<P>();   // lanes per row
  constexpr int RPB = NT / G;               // rows per workgroup step
  constexpr int NWV = NT / 64;               // wavefronts per workgroup
  constexpr int ST = col_stride<P>(16);
  constexpr int R1 = stage_radix<P, 1>();
  constexpr int NB1 = P / R1, PB1 = NB1 / G;
  static_assert(PB1 == 1 && RPB >= 1 && RPB * G == NT, "one first-stage butterfly per lane, whole rows per workgroup");
  constexpr int NSL = last_ns<P, 1>();
  constexpr int RL = stage_radix<P, NSL>();
  constexpr int PBL = (P / RL) / G;
  constexpr int ROUT = HALF ? RL / 2 : RL;
  constexpr int NOUT = PBL * ROUT;
  static_assert(NOUT <= 32, "output mask");
  static_assert(MODE == 0 || MODE == 1, "threshold or spectrum");
  __shared__ cx<T> lds[2 * RPB * ST];
  // per-wavefront candidate staging: (template of the launch, bin, 2F)
  __shared__ int st_item[NWV][STAGE_CAP];
  __shared__ int st_bin[NWV][STAGE_CAP];
  __shared__ float st_val[NWV][STAGE_CAP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = threadIdx.x / G, g = threadIdx.x % G;
  const int units = ta.Q / RPB;        // row units of one template
  const int total = ntmpl * units;     // row units of the launch
  const int nwg = gridDim.x;
  cx<T>* cola = lds + (2 * sub) * ST;
  cx<T>* colb = cola + ST;
  const T thr = (T)oa.threshold;
  const int search = oa.search_next[0] - 1;
  StageTw<T, P, G, R1> tw;
  tw.load(twst, g);
  const auto& twl = last_stage_tw<T, P, G, R1>(tw);

  // unit U of the launch: template U / units, rows (U % units) RPB + sub
  auto load_unit = [&](cx<T> (&ca)[PB1][R1], cx<T> (&cb)[PB1][R1], int U) {
    const int item = U / units, u = U - item * units;
    const cx<T>* p = tbuf + (long)(2 * item) * ta.L + 2 * (long)(u * RPB + sub) * P;
#pragma unroll
    for (int r = 0; r < R1; ++r) load_stream(p + 2 * (g + NB1 * r), ca[0][r], cb[0][r]);
  };

  WaveStage stg{st_item[wave], st_bin[wave], st_val[wave]};

  int U = blockIdx.x;
  if (U >= total) return;   // the same for the whole workgroup
  cx<T> xa[PB1][R1], xb[PB1][R1];
  load_unit(xa, xb, U);
  for (; U < total; U += nwg) {
    const int item = U / units;
    const int u = U - item * units;
    const int t = ta.t0 + item;
    const int skyl = t / ta.nfdot, sidx = t - skyl * ta.nfdot;
    const SkyParams& pr = sp[skyl];
    const T cfa = (T)pr.cfa, cfb = (T)pr.cfb, cfab = (T)pr.cfab;
    dftr<T, R1, false>(xa[0]);
    dftr<T, R1, false>(xb[0]);
    __syncthreads();  // the previous unit's last stage has read the tile
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xa, cola, g);
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xb, colb, g);
    __syncthreads();
    // the next unit's loads go into the registers just freed and overlap the rest
    if (U + nwg < total) load_unit(xa, xb, U + nwg);
    middle_stages_reg<T, P, G, R1, false>(cola, colb, g, tw);
    cx<T> fa[PBL][RL], fb[PBL][RL];
    stage_from_lds_reg<T, P, G, NSL, RL, PBL, HALF>(fa, cola, g, twl.w);
    stage_from_lds_reg<T, P, G, NSL, RL, PBL, HALF>(fb, colb, g, twl.w);
    const int k2 = u * RPB + sub;
    if constexpr (MODE == 1) {
      T* out = (T*)oa.spectrum + ((long)(ta.sky0 + skyl) * ta.nfdot + sidx) * (long)(oa.k_max - oa.k_min);
#pragma unroll
      for (int b = 0; b < PBL; ++b)
#pragma unroll
        for (int r = 0; r < ROUT; ++r) {
          const int k = ta.Q * (g + G * b + NSL * r) + k2;
          if (HALF || (k >= oa.k_min && k < oa.k_max))
            out[k - oa.k_min] = two_f_value(fa[b][r], fb[b][r], cfa, cfb, cfab);
        }
    } else {
      uint32_t mask = 0;
      T val[NOUT];
#pragma unroll
      for (int b = 0; b < PBL; ++b)
#pragma unroll
        for (int r = 0; r < ROUT; ++r) {
          const int k = ta.Q * (g + G * b + NSL * r) + k2;
          const T v = two_f_value(fa[b][r], fb[b][r], cfa, cfb, cfab);
          val[b * ROUT + r] = v;
          if ((HALF || (k >= oa.k_min && k < oa.k_max)) && v > thr) mask |= 1u << (b * ROUT + r);
        }
      stg.add<false>(oa, ta, search, lane, mask, val, item,
                     [&](int q) { return ta.Q * (g + G * (q / ROUT) + NSL * (q % ROUT)) + k2; });
    }
  }
  if constexpr (MODE == 0) stg.flush(oa, ta, search, lane);
}

// ---------------------------------------------------------------- pass B with interbinning (FP32)
// The template transforms have L = nfft/2 points.  Bin 2k of the nfft grid is bin k of the
// transform; bin 2k + 1 is w (X_k - X_{k+1 mod L}) for each series.  Bin k = Q k1 + k2 lies in
// row k2 of the intermediate and its neighbour k + 1 in row k2 + 1 at the same k1 (for row
// Q - 1: row 0 at k1 + 1).  A wavefront walks chunks of IB_CHUNK consecutive row units of
// one template (chunks w, w + nw, ... of the launch, so that the rows in flight form one
// window of HBM, as in k_tmpl_b_stream), and within a chunk the units in order: the
// neighbour of a lane's output is one row later, at lane + G in the same unit or, for the
// unit's last row, at lane g of the next unit's first row.  A unit's odd bins are formed
// once the next unit has been transformed; after a chunk's last unit the wavefront
// transforms one more, the next chunk's first unit or, at the template's end, the
// template's first unit (the neighbours k1 + 1 of row Q - 1).  Loads, stages and candidate
// staging are those of k_tmpl_b_stream.  With
// HALF (bins [0, nfft/2)) only the outputs k1 < P/2 are formed, plus output k1 = P/2 of the
// first butterfly, the neighbour of row Q - 1 at k1 = P/2 - 1.

// Flat output index o = b RO + r of a lane's outputs (k1 = g + G b + NSL r, r < RO).  For
// g = G - 1 the output holding k1 + 1 is in lane 0 at ib_next(o): the same r in the next
// butterfly, r + 1 in the first, or past the last (k1 + 1 = P/2 with HALF: the extra output
// NO; k1 + 1 = P otherwise: output 0, since the transform is periodic).
template <int PBL, int RO, int RL>
__host__ __device__ constexpr int ib_next(int o) {
  return (o / RO + 1 < PBL) ? o + RO : (o % RO + 1 < RO ? o % RO + 1 : (RO < RL ? PBL * RO : 0));
}

__device__ __forceinline__ cx<float> shfl_cx(cx<float> v, int src) {
  return mk<float>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

// dft_first_half plus output R/2: the alternating sum of the inputs.
template <typename T, int R>
__device__ __forceinline__ void dft_first_half_mid(cx<T>* v, cx<T>& mid) {
  if constexpr (R == 2) {
    mid = v[0] - v[1];
  } else if constexpr (R == 4) {
    mid = (v[0] + v[2]) - (v[1] + v[3]);
  } else {
    mid = ((v[0] + v[4]) + (v[2] + v[6])) - ((v[1] + v[5]) + (v[3] + v[7]));
  }
  dft_first_half<T, R>(v);
}

constexpr int IB_CHUNK = 16;

template <int P, int MODE, bool HALF>
__global__ void __launch_bounds__(256) k_tmpl_b_ib(TmplArgs ta, int ntmpl, const SkyParams* __restrict__ sp,
                                                   const cx<float>* __restrict__ tbuf, OutArgs oa,
                                                   const cx<float>* __restrict__ twst) {
  using T = float;
  constexpr int G = groups_per_col<P>();
  static_assert(G <= 64 && 64 % G == 0, "rows must tile a wavefront");
  constexpr int RPW = stream_rpw<P>();
  constexpr int ST = col_stride<P>(16);
  constexpr int R1 = stage_radix<P, 1>();
  constexpr int NB1 = P / R1, PB1 = NB1 / G;
  static_assert(PB1 >= 1 && NB1 % G == 0, "first stage must give each lane whole butterflies");
  constexpr int NSL = last_ns<P, 1>();
  constexpr int RL = stage_radix<P, NSL>();
  constexpr int PBL = (P / RL) / G;
  constexpr int RO = HALF ? RL / 2 : RL;       // outputs kept per last-stage butterfly
  constexpr int NO = PBL * RO;                 // outputs per lane and series
  constexpr int NX = HALF ? NO + 1 : NO;       // plus output P/2 of the first butterfly
  constexpr int NV = 2 * NO;                   // 2F values per lane and unit: even and odd bins
  static_assert(NV <= 32, "output mask");
  __shared__ cx<T> lds[4 * 2 * RPW * ST];
  __shared__ int st_item[4][STAGE_CAP];
  __shared__ int st_bin[4][STAGE_CAP];
  __shared__ float st_val[4][STAGE_CAP];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int units = ta.Q / RPW;                 // row units of one template (a power of two)
  const int ch = units < IB_CHUNK ? units : IB_CHUNK;
  const int lg_cpt = __builtin_ctz((unsigned)(units / ch));   // chunks per template, log2
  const int nchunk = ntmpl << lg_cpt;           // chunks of the launch
  const int nw = gridDim.x * 4;                 // wavefronts of the grid
  int c = blockIdx.x * 4 + wave;
  if (c >= nchunk) return;
  const int sub = lane / G, g = lane % G;
  cx<T>* cola = lds + (wave * 2 * RPW + sub) * ST;
  cx<T>* colb = cola + RPW * ST;
  const T thr = (T)oa.threshold;
  const T wib = ta.ibw;
  const int search = oa.search_next[0] - 1;
  StageTw<T, P, G, R1> tw;
  tw.load(twst, g);
  const auto& twl = last_stage_tw<T, P, G, R1>(tw);
  const int lofs = sub * P + g;

  auto load_unit = [&](cx<T> (&ca)[PB1][R1], cx<T> (&cb)[PB1][R1], int item, int u) {
    const cx<T>* p = tbuf + 2 * (long)item * ta.L + 2 * (long)u * (RPW * P);
#pragma unroll
    for (int b = 0; b < PB1; ++b)
#pragma unroll
      for (int r = 0; r < R1; ++r) load_stream(p + 2 * (lofs + G * b + NB1 * r), ca[b][r], cb[b][r]);
  };

  // last stage: the kept outputs of every butterfly in flat order (and output P/2 of the first)
  auto last_stage = [&](cx<T>* col, cx<T> (&f)[NX]) {
    constexpr int NB = P / RL;
    static_assert(NB % 8 == 0, "constant offsets need NB a multiple of 8");
    const cx<T>* p = col + phys(g);
#pragma unroll
    for (int b = 0; b < PBL; ++b) {
      cx<T> v[RL];
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int c = G * b + r * NB;
        cx<T> x = p[c + c / 8];
        if (r > 0) x = cmul(x, twl.w[b][r - 1]);
        v[r] = x;
      }
      if constexpr (HALF) {
        if (b == 0) dft_first_half_mid<T, RL>(v, f[NO]);
        else dft_first_half<T, RL>(v);
      } else {
        dftr<T, RL, false>(v);
      }
#pragma unroll
      for (int r = 0; r < RO; ++r) f[b * RO + r] = v[r];
    }
  };

  WaveStage stg{st_item[wave], st_bin[wave], st_val[wave]};

  // Even and odd bins of unit V (outputs pa, pb) with the neighbours of its rows in the unit
  // just transformed (outputs fa, fb); `wrap`: that unit is the template's first unit again.
  cx<T> pa[NO], pb[NO];
  int c_item = -1, skyl = 0, sidx = 0;   // template of the cached constants
  T cfa = 0, cfb = 0, cfab = 0;
  auto finish = [&](int item, int u, bool wrap, const cx<T> (&fa)[NX], const cx<T> (&fb)[NX]) {
    if (item != c_item) {
      c_item = item;
      const int t = ta.t0 + item;
      skyl = t / ta.nfdot;
      sidx = t - skyl * ta.nfdot;
      const SkyParams& pr = sp[skyl];
      cfa = (T)pr.cfa;
      cfb = (T)pr.cfb;
      cfab = (T)pr.cfab;
    }
    const int k2 = u * RPW + sub;
    // Neighbours by lane shuffles.  The only reader of lane 0's current outputs is lane
    // (RPW - 1, G - 1) when `wrap` (it needs output ib_next(o) there) and lane (RPW - 1, 0)
    // otherwise, so lane 0 supplies whichever is wanted.
    const bool inner = sub < RPW - 1;
    const int src = inner ? lane + G : (wrap ? (g + 1) % G : g);
    T val[NV];
    auto two_f = [&](cx<T> a, cx<T> b, auto cross_c) {
      if constexpr (decltype(cross_c)::value) return two_f_value(a, b, cfa, cfb, cfab);
      else return two_f_value_nc(a, b, cfa, cfb);
    };
    auto values = [&](auto cross_c) {
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      cx<T> na, nb;
      if (RPW == 1 && !wrap) {
        na = fa[o];
        nb = fb[o];
      } else {
        const bool alt = wrap && lane == 0;
        const int on = ib_next<PBL, RO, RL>(o);   // a constant once the loop is unrolled
        const cx<T> sa = alt ? fa[on] : fa[o];
        const cx<T> sb = alt ? fb[on] : fb[o];
        na = shfl_cx(sa, src);
        nb = shfl_cx(sb, src);
        if constexpr (RPW > 1) {
          const cx<T> qa = shfl_cx(pa[o], src), qb = shfl_cx(pb[o], src);
          na = inner ? qa : na;
          nb = inner ? qb : nb;
        }
      }
      val[2 * o] = two_f(pa[o], pb[o], cross_c);
      const cx<T> da = pa[o] - na, db = pb[o] - nb;
      val[2 * o + 1] = two_f(mk<T>(wib * da.re, wib * da.im), mk<T>(wib * db.re, wib * db.im), cross_c);
    }
    };
    if (cfab != (T)0) values(std::true_type{});
    else values(std::false_type{});
    auto bin_of = [&](int v) {
      const int o = v >> 1;
      return 2 * (ta.Q * (g + G * (o / RO) + NSL * (o % RO)) + k2) + (v & 1);
    };
    if constexpr (MODE == 1) {
      T* out = (T*)oa.spectrum + ((long)(ta.sky0 + skyl) * ta.nfdot + sidx) * (long)(oa.k_max - oa.k_min);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int k = bin_of(v);
        if (HALF || (k >= oa.k_min && k < oa.k_max)) out[k - oa.k_min] = val[v];
      }
    } else {
      float* srow = (float*)oa.spectrum + (long)item * (long)(oa.k_max - oa.k_min);
      uint32_t mask = 0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int k = bin_of(v);
        const bool inr = HALF || (k >= oa.k_min && k < oa.k_max);
        if (MODE == 2 && inr) srow[k - oa.k_min] = (float)val[v];
        if (inr && val[v] > thr) mask |= 1u << v;
      }
      stg.add<true>(oa, ta, search, lane, mask, val, item, bin_of);
    }
  };

  // The walk: step j = 0 .. ch of chunk c transforms unit u0 + j of template item (step ch:
  // the unit after the chunk, unit 0 at the template's end) and forms the bins of unit
  // u0 + j - 1.
  auto unit_of = [&](int u0, int j) { return j < ch ? u0 + j : (u0 + ch == units ? 0 : u0 + ch); };
  int item = c >> lg_cpt, u0 = (c - (item << lg_cpt)) * ch, j = 0;
  cx<T> xa[PB1][R1], xb[PB1][R1];
  load_unit(xa, xb, item, u0);
  while (true) {
#pragma unroll
    for (int b = 0; b < PB1; ++b) {
      dftr<T, R1, false>(xa[b]);
      dftr<T, R1, false>(xb[b]);
    }
    stage_sync<true>();  // the previous unit's last stage has read the slab
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xa, cola, g);
    stage_to_lds_off<T, P, G, 1, R1, PB1>(xb, colb, g);
    stage_sync<true>();
    int n_c = c, n_item = item, n_u0 = u0, n_j = j + 1;
    if (j == ch) {
      n_c = c + nw;
      n_item = n_c >> lg_cpt;
      n_u0 = (n_c - (n_item << lg_cpt)) * ch;
      n_j = 0;
    }
    const bool more = n_c < nchunk;
    if (more) load_unit(xa, xb, n_item, unit_of(n_u0, n_j));
    middle_stages_reg<T, P, G, R1>(cola, colb, g, tw);
    cx<T> fa[NX], fb[NX];
    last_stage(cola, fa);
    last_stage(colb, fb);
    if (j > 0) finish(item, u0 + j - 1, j == ch && u0 + ch == units, fa, fb);
    if (j < ch) {
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        pa[o] = fa[o];
        pb[o] = fb[o];
      }
    }
    if (!more) break;
    c = n_c;
    item = n_item;
    u0 = n_u0;
    j = n_j;
  }
  if constexpr (MODE != 1) stg.flush(oa, ta, search, lane);
}

// Count of candidates before a launch (read by the patch capture after it).
__global__ void k_record_count(const unsigned long long* __restrict__ count, unsigned long long* __restrict__ first) {
  if (threadIdx.x == 0 && blockIdx.x == 0) first[0] = count[0];
}

// For each candidate slot written by the launch ([first, min(count, capacity))), copy
// the 2F window [bin - 128, bin + 128) of its template from the launch's spectrum rows
// into patches[slot]; bins outside [k_min, k_max) read 0.  One workgroup (256 threads)
// per patch, grid-stride over the slots.
__global__ void __launch_bounds__(256) k_capture_patches(const CandEntry* __restrict__ cand,
                                                         const float* __restrict__ spec, float* __restrict__ patches,
                                                         unsigned long long patch_capacity,
                                                         const unsigned long long* __restrict__ count,
                                                         const unsigned long long* __restrict__ first, int k_min,
                                                         int k_max, int t0, int nfdot, int sky0, int tq, int trow) {
  unsigned long long end = count[0];
  if (end > patch_capacity) end = patch_capacity;
  // rows of bins [k_min, k_max) per template, or (tq > 0) the rows of the streaming
  // second pass: tq rows of trow values in blocks of CAP_BLOCK columns, bin k at row
  // k % tq, column k / tq, [column / CAP_BLOCK][row][column % CAP_BLOCK]
  const long tlen = tq > 0 ? (long)tq * trow : (long)(k_max - k_min);
  for (unsigned long long slot = first[0] + blockIdx.x; slot < end; slot += gridDim.x) {
    const CandEntry ce = cand[slot];
    const long t_local = (long)(ce.sky - sky0) * nfdot + ce.fdot_idx - t0;
    const int k = ce.bin - 128 + (int)threadIdx.x;
    float v = 0.f;
    if (k >= k_min && k < k_max)
      v = spec[t_local * tlen + (tq > 0 ? (long)(k / tq / CAP_BLOCK) * tq * CAP_BLOCK + (long)(k % tq) * CAP_BLOCK +
                                             (k / tq) % CAP_BLOCK
                                           : (long)(k - k_min))];
    patches[slot * 256 + threadIdx.x] = v;
  }
}

}  // namespace fstat

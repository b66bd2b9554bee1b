// Candidate drain on the device: the entries emitted in arbitrary order (atomics) are put
// into key order (search, segment, sky, spindown index, bin) before they are copied out.
// Count -> offsets -> write, as the paper's candidate output is organised (Sect. 3.2):
//   1. count the entries of every template (one atomic per entry, which also gives the
//      entry its rank among its template's entries in arrival order);
//   2. exclusive scan of the counts: each template's offset in the output;
//   3. write every entry to its template's range (template order);
//   4. order each template's range by bin (bins within a template are distinct, so an
//      entry's place is the number of entries of its template with a smaller bin);
//   5. form the records and keys for the copy out.
// Templates are numbered search by search (searches since the previous drain), then
// segment, sky, spindown: t = base[search] + (segment * nsky + sky) * nfdot + fdot_idx.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fstat_kernels.hpp"

namespace fstat {

struct DrainSearch {
  long long base;     // number of the search's first template
  int nsky, nfdot;
};

constexpr int DRAIN_NT = 256;
constexpr int SCAN_TILE = 4096;                 // counts per workgroup of the scan (16 per thread)
constexpr int DRAIN_SEG_MAX = 4096;             // longest template range ordered by counting (longer: bitmap)

__device__ __forceinline__ long long drain_template(const CandEntry& c, const DrainSearch* __restrict__ s,
                                                    int nsearch, int search0, int nseg, unsigned* bad) {
  const int r = c.search - search0;
  if (r < 0 || r >= nsearch) {
    atomicOr(bad, 1u);
    return -1;
  }
  const DrainSearch d = s[r];
  if (c.segment < 0 || c.segment >= nseg || c.sky < 0 || c.sky >= d.nsky || c.fdot_idx < 0 || c.fdot_idx >= d.nfdot) {
    atomicOr(bad, 1u);
    return -1;
  }
  return d.base + ((long long)c.segment * d.nsky + c.sky) * d.nfdot + c.fdot_idx;
}

__global__ void k_drain_zero(unsigned* __restrict__ a, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    a[i] = 0u;
}

// 1. per-template counts; rank[i] = the entry's place among its template's entries so far
__global__ void k_drain_count(const CandEntry* __restrict__ cand, long long n, const DrainSearch* __restrict__ s,
                              int nsearch, int search0, int nseg, unsigned* __restrict__ counts,
                              unsigned* __restrict__ rank, unsigned* bad) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const long long t = drain_template(cand[i], s, nsearch, search0, nseg, bad);
    rank[i] = t < 0 ? 0u : atomicAdd(&counts[t], 1u);
  }
}

// Sum of 16 consecutive counts per thread, then of the workgroup's 4096.
__device__ __forceinline__ unsigned long long tile_thread_sum(const unsigned* __restrict__ a, long long n,
                                                              long long i0) {
  unsigned long long v = 0;
  for (int k = 0; k < SCAN_TILE / DRAIN_NT; ++k) {
    const long long i = i0 + k;
    if (i < n) v += a[i];
  }
  return v;
}

// Inclusive scan over the workgroup of one 64-bit value per thread (wavefront shuffles,
// then the wavefront totals through LDS); *total gets the workgroup's sum.
__device__ __forceinline__ unsigned long long block_inclusive_scan_u64(unsigned long long v,
                                                                       unsigned long long* total) {
  __shared__ unsigned long long wsum[DRAIN_NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  if (lane == 63) wsum[wv] = v;
  __syncthreads();
  unsigned long long before = 0, all = 0;
  for (int w = 0; w < DRAIN_NT / 64; ++w) {
    if (w < wv) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return v + before;
}

// 2a. workgroup sums of tiles of SCAN_TILE counts
__global__ void __launch_bounds__(DRAIN_NT) k_scan_tile_sums(const unsigned* __restrict__ a, long long n,
                                                             unsigned long long* __restrict__ sums) {
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * (SCAN_TILE / DRAIN_NT);
  unsigned long long tot;
  (void)block_inclusive_scan_u64(tile_thread_sum(a, n, base), &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// 2b. exclusive scan of the tile sums in place, by one workgroup walking them in order
__global__ void __launch_bounds__(DRAIN_NT) k_scan_sums(unsigned long long* __restrict__ sums, long long ntiles) {
  unsigned long long carry = 0;
  for (long long j0 = 0; j0 < ntiles; j0 += DRAIN_NT) {
    const long long j = j0 + threadIdx.x;
    const unsigned long long v = j < ntiles ? sums[j] : 0ull;
    unsigned long long tot;
    const unsigned long long inc = block_inclusive_scan_u64(v, &tot);
    if (j < ntiles) sums[j] = carry + inc - v;
    carry += tot;
  }
}

// 2c. off[i] = sum of counts before i (i < n), off[n] = the total: each workgroup scans its tile
__global__ void __launch_bounds__(DRAIN_NT) k_scan_apply(const unsigned* __restrict__ a, long long n,
                                                         const unsigned long long* __restrict__ sums,
                                                         unsigned long long* __restrict__ off) {
  constexpr int PER = SCAN_TILE / DRAIN_NT;
  const long long i0 = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * PER;
  unsigned long long tot;
  const unsigned long long own = tile_thread_sum(a, n, i0);
  unsigned long long run = sums[blockIdx.x] + block_inclusive_scan_u64(own, &tot) - own;
  for (int k = 0; k < PER; ++k) {
    const long long i = i0 + k;
    if (i < n) {
      off[i] = run;
      run += a[i];
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == DRAIN_NT - 1) off[n] = sums[blockIdx.x] + tot;
}

// 3. every entry to its template's range, in arrival order
__global__ void k_drain_scatter(const CandEntry* __restrict__ cand, long long n, const DrainSearch* __restrict__ s,
                                int nsearch, int search0, int nseg, const unsigned long long* __restrict__ off,
                                const unsigned* __restrict__ rank, CandEntry* __restrict__ grouped, unsigned* bad) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const CandEntry c = cand[i];
    const long long t = drain_template(c, s, nsearch, search0, nseg, bad);
    if (t >= 0) grouped[off[t] + rank[i]] = c;
  }
}

// 4. each template's range ordered by bin, one workgroup per template (grid-stride over
// templates).  Ranges of at most DRAIN_SEG_MAX entries: an entry's place is the number of
// entries of its template with a smaller bin (the bins in LDS); longer ranges are left to
// k_drain_order_long.
__global__ void __launch_bounds__(DRAIN_NT) k_drain_order(const CandEntry* __restrict__ grouped,
                                                          const unsigned long long* __restrict__ off, long long ntpl,
                                                          CandEntry* __restrict__ out) {
  __shared__ int sbin[DRAIN_SEG_MAX];
  for (long long t = blockIdx.x; t < ntpl; t += gridDim.x) {
    const unsigned long long a = off[t], c = off[t + 1] - a;
    if (c == 0 || c > (unsigned long long)DRAIN_SEG_MAX) continue;
    const int m = (int)c;
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += DRAIN_NT) sbin[j] = grouped[a + j].bin;
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += DRAIN_NT) {
      const int b = sbin[j];
      int r = 0;
      for (int k = 0; k < m; ++k) r += (sbin[k] < b) | ((sbin[k] == b) & (k < j));
      out[a + r] = grouped[a + j];
    }
  }
}

// 4b. ranges longer than DRAIN_SEG_MAX (thresholds low enough that a good share of a
// template's bins cross): a bitmap of the template's bins in LDS (up to 2^20 bins, the
// longest transform), popcounts of 32-word blocks scanned across the workgroup, and each
// entry's place = the set bits below its bin.  Bins of one template are distinct: a
// repeated one, or a range wider than the bitmap, sets *bad.
constexpr int DRAIN_LONG_NT = 1024;
constexpr int DRAIN_BITMAP_WORDS = (1 << 20) / 32;
__global__ void __launch_bounds__(DRAIN_LONG_NT) k_drain_order_long(const CandEntry* __restrict__ grouped,
                                                                    const unsigned long long* __restrict__ off,
                                                                    long long ntpl, CandEntry* __restrict__ out,
                                                                    unsigned* bad) {
  __shared__ unsigned bits[DRAIN_BITMAP_WORDS];
  __shared__ unsigned bpre[DRAIN_BITMAP_WORDS / 32];
  __shared__ int rmin[DRAIN_LONG_NT / 64], rmax[DRAIN_LONG_NT / 64];
  __shared__ unsigned wsum[DRAIN_LONG_NT / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (long long t = blockIdx.x; t < ntpl; t += gridDim.x) {
    const unsigned long long a = off[t], c = off[t + 1] - a;
    if (c <= (unsigned long long)DRAIN_SEG_MAX) continue;
    // the template's bin range
    int lo = 0x7fffffff, hi = -0x7fffffff - 1;
    for (unsigned long long j = tid; j < c; j += DRAIN_LONG_NT) {
      const int b = grouped[a + j].bin;
      lo = min(lo, b);
      hi = max(hi, b);
    }
    for (int d = 32; d >= 1; d >>= 1) {
      lo = min(lo, __shfl_xor(lo, d, 64));
      hi = max(hi, __shfl_xor(hi, d, 64));
    }
    __syncthreads();   // the previous template's readers of the shared arrays are done
    if (lane == 0) {
      rmin[wv] = lo;
      rmax[wv] = hi;
    }
    __syncthreads();
    lo = rmin[0];
    hi = rmax[0];
    for (int k = 1; k < DRAIN_LONG_NT / 64; ++k) {
      lo = min(lo, rmin[k]);
      hi = max(hi, rmax[k]);
    }
    if ((long long)hi - lo >= (long long)DRAIN_BITMAP_WORDS * 32) {
      if (tid == 0) atomicOr(bad, 1u);
      continue;
    }
    const int nw = ((hi - lo) >> 5) + 1, nb = (nw + 31) >> 5;
    for (int w = tid; w < nw; w += DRAIN_LONG_NT) bits[w] = 0u;
    __syncthreads();
    for (unsigned long long j = tid; j < c; j += DRAIN_LONG_NT) {
      const int d = grouped[a + j].bin - lo;
      const unsigned m = 1u << (d & 31);
      if (atomicOr(&bits[d >> 5], m) & m) atomicOr(bad, 1u);
    }
    __syncthreads();
    // exclusive scan of the 32-word blocks' popcounts (one block per thread, nb <= 1024)
    unsigned v = 0;
    if (tid < nb)
      for (int k = 0; k < 32; ++k) {
        const int w = tid * 32 + k;
        if (w < nw) v += __popc(bits[w]);
      }
    unsigned inc = v;
    for (int d = 1; d < 64; d <<= 1) {
      const unsigned u = __shfl_up(inc, d, 64);
      if (lane >= d) inc += u;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    unsigned before = 0;
    for (int k = 0; k < wv; ++k) before += wsum[k];
    if (tid < nb) bpre[tid] = before + inc - v;
    __syncthreads();
    for (unsigned long long j = tid; j < c; j += DRAIN_LONG_NT) {
      const CandEntry e = grouped[a + j];
      const int d = e.bin - lo, w = d >> 5;
      unsigned r = bpre[w >> 5];
      for (int u = w & ~31; u < w; ++u) r += __popc(bits[u]);
      r += __popc(bits[w] & ((1u << (d & 31)) - 1u));
      out[a + r] = e;
    }
  }
}

// 5. the records and keys of the ordered entries, formed as the host would form them (the
// paper's five numbers from the search's lists, the integer key, the vetting score), for a
// copy straight into the caller's arrays
struct DrainList {
  const double* v;   // device copy: alpha[nsky], delta[nsky], then fdot[nfdot] (explicit
                     // list) or w_freq[nsky], w_spin[nsky] (lattice grid)
  int nsky, lattice, s_lo;
  double m10, m11;
};
struct DrainSeg {
  double f_off, dt;
  int nfft;
};

__global__ void k_drain_records(const CandEntry* __restrict__ ent, long long n, const DrainList* __restrict__ lists,
                                int search0, const DrainSeg* __restrict__ segs, int scored,
                                fstat_candidate* __restrict__ out, fstat_candidate_key* __restrict__ keys) {
#pragma clang fp contract(off)
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const CandEntry c = ent[i];
    if (keys) {
      fstat_candidate_key k;
      k.search = c.search;
      k.segment = c.segment;
      k.sky = c.sky;
      k.fdot_idx = c.fdot_idx;
      k.bin = c.bin;
      k.vet_score = scored ? __int_as_float(c.pad) : __builtin_nanf("");
      keys[i] = k;
    }
    if (out) {
      const DrainList& L = lists[c.search - search0];
      const DrainSeg sg = segs[c.segment];
      fstat_candidate r;
      if (L.lattice) {
        // the template's frequency shift and spindown, as the search kernels formed them
        const int s = L.s_lo + c.fdot_idx;
        const double u = lattice_shift_bins(lattice_w(s, L.m10, L.v[2 * L.nsky + c.sky]), (double)sg.nfft / (2.0 * M_PI));
        r.f_hz = sg.f_off + ((double)c.bin + u) / ((double)sg.nfft * sg.dt);
        r.fdot = lattice_w(s, L.m11, L.v[3 * L.nsky + c.sky]) / (M_PI * sg.dt * sg.dt);
      } else {
        r.f_hz = sg.f_off + (double)c.bin / ((double)sg.nfft * sg.dt);
        r.fdot = L.v[2 * L.nsky + c.fdot_idx];
      }
      r.alpha = L.v[c.sky];
      r.delta = L.v[L.nsky + c.sky];
      r.twoF = c.twoF;
      out[i] = r;
    }
  }
}

}  // namespace fstat

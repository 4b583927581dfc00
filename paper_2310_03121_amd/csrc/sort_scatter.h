// The species sort and scatter as one block's work (blocks blk of nblk
// staging blocks, 256 threads), shared by the sort kernel and the launch that
// runs the sort beside the molecule neighbor search.
#pragma once
#include "kernels.h"

namespace nnp {

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// For up to kFusedSortBlocks staging blocks: every block sums the staging
// histograms itself (totals, and its own prefix over earlier blocks), so no
// separate scan kernel is needed; block 0 also writes the group table, the
// pad-row markers and the staging bits of the status word, as k_groups does.
// Rows are the same as with k_groups + k_scatter.
__device__ __forceinline__ void sort_scatter_block(int blk, int nblk, const int* __restrict__ dims,
                                                   int S, const float4* __restrict__ xyzs,
                                                   const int* __restrict__ hist,
                                                   GroupTable* __restrict__ gt,
                                                   int* __restrict__ row, int* __restrict__ perm,
                                                   int rows_cap, const int* __restrict__ off,
                                                   int wchunk_rows,
                                                   uint32_t* __restrict__ status) {
  __shared__ int tot[kMaxS], pre[kMaxS], pst[kMaxS + 1];
  __shared__ int wcnt[4][kMaxS];
  __shared__ unsigned int bits_all;
  const int n = dims[0], nmol = dims[1];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) bits_all = 0u;
  for (int q = w; q < kMaxS; q += 4) {
    int all = 0, before = 0;
    if (q < S)
      for (int b = lane; b < nblk; b += kWave) {
        const int v = hist[q * nblk + b];
        all += v;
        before += b < blk ? v : 0;
      }
    all = wave_sum_i(all);
    before = wave_sum_i(before);
    if (lane == 0) {
      tot[q] = all;
      pre[q] = before;
    }
  }
  __syncthreads();
  if (t == 0) {
    int p = 0, c = 0;
    for (int q = 0; q < kMaxS; ++q) {
      const int cnt = q < S ? tot[q] : 0;
      pst[q] = p;
      if (blk == 0) {
        gt->cnt[q] = cnt;
        gt->pstart[q] = p;
        gt->wchunk[q] = c;
      }
      p += (cnt + kPad - 1) / kPad * kPad;
      c += (cnt + wchunk_rows - 1) / wchunk_rows;
    }
    pst[kMaxS] = p;
    if (blk == 0) {
      gt->pstart[kMaxS] = p;
      gt->wchunk[kMaxS] = c;
      gt->total_rows = p;
      gt->n_wchunks = c;
    }
  }
  __syncthreads();
  // stable scatter: rank = group start + earlier blocks + earlier waves of
  // this block + earlier lanes of the wave with the same species
  const int i = blk * blockDim.x + t;
  const int s = i < n ? species_of(xyzs[i]) : -1;
  int rank = 0;
  for (int q = 0; q < S; ++q) {
    uint64_t m = ballot(s == q);
    if (s == q) rank = popc_below(m);
    if (lane == 0) wcnt[w][q] = __popcll(m);
  }
  __syncthreads();
  if (i < n) {
    int base = pst[s] + pre[s];
    for (int v = 0; v < w; ++v) base += wcnt[v][s];
    const int r = base + rank;
    row[i] = r;
    perm[r] = i;
  }
  if (blk != 0) return;
  // block 0: pad rows, offsets, staging error bits
  for (int q = 0; q < kMaxS; ++q) {
    const int a = pst[q] + (q < S ? tot[q] : 0), e = pst[q + 1];
    for (int r = a + t; r < e; r += blockDim.x) perm[r] = -1;
  }
  for (int r = pst[kMaxS] + t; r < rows_cap; r += blockDim.x) perm[r] = -1;
  bool bad = false;
  for (int m = t; m < nmol; m += blockDim.x) bad |= off[m] > off[m + 1];
  if (t == 0) bad |= off[0] != 0 || off[nmol] != n;
  uint32_t bits = bad ? kStOffsets : 0u;
  for (int b = t; b < nblk; b += blockDim.x) bits |= (uint32_t)hist[kMaxS * nblk + b];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) bits |= (uint32_t)__shfl_xor((int)bits, o, 64);
  if (lane == 0 && bits) atomicOr(&bits_all, bits);
  __syncthreads();
  if (t == 0 && bits_all) atomicOr(status, bits_all);
}

}  // namespace nnp

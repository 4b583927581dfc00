// Staging, species sort and energy reduction.
//
// Staging turns the caller's AoS float32 positions into float4 records
// (x, y, z, species bits), finds each atom's molecule from the offsets, zeroes
// the force output, validates species and positions, and histograms species
// per block.  The species sort is a stable counting sort: every species group
// starts at a multiple of kPad rows, so the per-element network GEMMs can tile
// rows without a tile straddling two elements (one network per element,
// Methods "OpenMM-ML").  The molecular energy is the FP64 sum of the FP32
// atomic energies plus self energies.
#include "kernels.h"

namespace nnp {

__global__ __launch_bounds__(256) void k_stage(int n_arg, int nmol_arg, int* __restrict__ dims,
                                               const float* __restrict__ pos,
                                               const double* __restrict__ pos64,
                                               const int* __restrict__ gidx, int n_total,
                                               const int* __restrict__ species,
                                               const int* __restrict__ off, int S,
                                               float4* __restrict__ xyzs, int* __restrict__ mol,
                                               float* __restrict__ Fzero, int* __restrict__ hist,
                                               uint32_t* __restrict__ status) {
  __shared__ int h[kMaxS];
  __shared__ uint32_t bits;
  const int n = n_arg >= 0 ? n_arg : dims[0];
  const int nmol = nmol_arg >= 0 ? nmol_arg : dims[1];
  if (blockIdx.x == 0 && threadIdx.x == 0 && n_arg >= 0) {
    dims[0] = n;
    dims[1] = nmol;
  }
  if (threadIdx.x < kMaxS) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) bits = 0;
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float x, y, z;
    uint32_t st = 0;
    int g = i;  // row of the position arrays
    if (gidx) {  // subset of a larger system: gather by index
      g = gidx[i];
      if (g < 0 || g >= n_total) {
        st |= kStOffsets;
        g = 0;
      }
    }
    if (pos64) {  // MD state: the potential sees the FP32 rounding of x
      x = (float)pos64[3 * g];
      y = (float)pos64[3 * g + 1];
      z = (float)pos64[3 * g + 2];
    } else {
      x = pos[3 * g];
      y = pos[3 * g + 1];
      z = pos[3 * g + 2];
    }
    int s = species[i];
    if (s < 0 || s >= S) {
      st |= kStSpecies;
      s = clampi(s, S);
    }
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
      st |= kStNonFinite;
      x = y = z = 0.f;
    }
    // molecule: the last m with off[m] <= i (off is non-decreasing when valid)
    int lo = 0, hi = nmol;
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid; else hi = mid;
    }
    mol[i] = lo;
    xyzs[i] = make_float4(x, y, z, __int_as_float(s));
    if (Fzero) {
      Fzero[3 * i] = 0.f;
      Fzero[3 * i + 1] = 0.f;
      Fzero[3 * i + 2] = 0.f;
    }
    atomicAdd(&h[s], 1);
    if (st) atomicOr(&bits, st);
  }
  __syncthreads();
  if (threadIdx.x < S) hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
  // this block's error bits; the group kernel folds them into the status word
  if (threadIdx.x == 0) hist[kMaxS * gridDim.x + blockIdx.x] = (int)bits;
}

// One block of kMaxS waves (wave q works on species q): species totals,
// padded group starts, per-block bases of the stable scatter (wave-level
// prefix sums, no block barriers inside the scans), pad-row markers,
// molecule-offset validation, the chunk table of the weight-gradient
// reduction, and the evaluation's status word (overwritten here; kernels
// that run later only add bits).
__global__ __launch_bounds__(512) void k_groups(const int* __restrict__ dims, int nblk, int S,
                                                int* __restrict__ hist, GroupTable* __restrict__ gt,
                                                int* __restrict__ perm, int rows_cap,
                                                const int* __restrict__ off, int wchunk_rows,
                                                uint32_t* __restrict__ status) {
  __shared__ int tot[kMaxS];
  __shared__ int pst[kMaxS + 1];
  __shared__ unsigned int bits_all;
  const int n = dims[0], nmol = dims[1];
  const int t = threadIdx.x, wq = t >> 6, lane = t & 63;
  if (t == 0) bits_all = 0u;
  if (wq < kMaxS) {
    int acc = 0;
    if (wq < S)
      for (int b = lane; b < nblk; b += kWave) acc += hist[wq * nblk + b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) tot[wq] = acc;
  }
  __syncthreads();
  if (t == 0) {
    int p = 0, c = 0;
    for (int q = 0; q < kMaxS; ++q) {
      const int cnt = q < S ? tot[q] : 0;
      pst[q] = p;
      gt->cnt[q] = cnt;
      gt->pstart[q] = p;
      gt->wchunk[q] = c;
      p += (cnt + kPad - 1) / kPad * kPad;
      c += (cnt + wchunk_rows - 1) / wchunk_rows;
    }
    pst[kMaxS] = p;
    gt->pstart[kMaxS] = p;
    gt->wchunk[kMaxS] = c;
    gt->total_rows = p;
    gt->n_wchunks = c;
  }
  __syncthreads();
  // exclusive scan of each species' block counts, offset by the group start
  if (wq < S) {
    int carry = pst[wq];
    for (int b0 = 0; b0 < nblk; b0 += kWave) {
      const int b = b0 + lane;
      const int v = b < nblk ? hist[wq * nblk + b] : 0;
      int incl = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
      }
      if (b < nblk) hist[wq * nblk + b] = carry + incl - v;
      carry += __shfl(incl, 63, 64);
    }
  }
  // pad rows: inside each group after its atoms, and after the last group
  for (int q = 0; q < kMaxS; ++q) {
    const int a = pst[q] + (q < S ? tot[q] : 0), e = pst[q + 1];
    for (int r = a + t; r < e; r += blockDim.x) perm[r] = -1;
  }
  for (int r = pst[kMaxS] + t; r < rows_cap; r += blockDim.x) perm[r] = -1;
  // offsets: off[0] == 0, non-decreasing, off[nmol] == n; staging bits
  bool bad = false;
  for (int m = t; m < nmol; m += blockDim.x) bad |= off[m] > off[m + 1];
  if (t == 0) bad |= off[0] != 0 || off[nmol] != n;
  uint32_t bits = bad ? kStOffsets : 0u;
  for (int b = t; b < nblk; b += blockDim.x) bits |= (uint32_t)hist[kMaxS * nblk + b];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) bits |= (uint32_t)__shfl_xor((int)bits, o, 64);
  if (lane == 0 && bits) atomicOr(&bits_all, bits);
  __syncthreads();
  if (t == 0) *status = bits_all;
}

// Stable scatter into species-sorted rows: rank = block base + earlier waves
// of the block + earlier lanes of the wave with the same species.
__global__ __launch_bounds__(256) void k_scatter(const int* __restrict__ dims, int S,
                                                 const float4* __restrict__ xyzs,
                                                 const int* __restrict__ hist, int* __restrict__ row,
                                                 int* __restrict__ perm) {
  __shared__ int wcnt[4][kMaxS];
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = threadIdx.x >> 6;
  const int s = i < n ? species_of(xyzs[i]) : -1;
  int rank = 0;
  for (int q = 0; q < S; ++q) {
    uint64_t m = ballot(s == q);
    if (s == q) rank = popc_below(m);
    if (lane_id() == 0) wcnt[w][q] = __popcll(m);
  }
  __syncthreads();
  if (i < n) {
    int base = hist[s * gridDim.x + blockIdx.x];
    for (int v = 0; v < w; ++v) base += wcnt[v][s];
    int r = base + rank;
    row[i] = r;
    perm[r] = i;
  }
}

// The species sort and scatter in one launch, for up to kFusedSortBlocks
// staging blocks: every block sums the staging histograms itself (totals,
// and its own prefix over earlier blocks), so no separate scan kernel is
// needed; block 0 also writes the group table, the pad-row markers and the
// status word, as k_groups does.  Rows are the same as with k_groups +
// k_scatter.
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(256) void k_sort_scatter(const int* __restrict__ dims, int S,
                                                      const float4* __restrict__ xyzs,
                                                      const int* __restrict__ hist,
                                                      GroupTable* __restrict__ gt,
                                                      int* __restrict__ row, int* __restrict__ perm,
                                                      int rows_cap, const int* __restrict__ off,
                                                      int wchunk_rows, uint32_t* __restrict__ status) {
  __shared__ int tot[kMaxS], pre[kMaxS], pst[kMaxS + 1];
  __shared__ int wcnt[4][kMaxS];
  __shared__ unsigned int bits_all;
  const int nblk = gridDim.x, blk = blockIdx.x;
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
  if (t == 0) *status = bits_all;
}

// One workgroup per molecule: E_m = sum_i (e_i + e_self[s_i]) with the
// atomic energies in input atom order; for an ensemble of M members e_i is
// the mean of the members' atomic energies (member k at eatom + k * mstride).
// Thread t sums the atoms t, t + 256, ... of the molecule (counted from its
// first atom), then the waves and the four wave sums combine in a fixed
// order: the result depends only on the molecule's own atoms, not on where
// it sits in a batch.
__global__ __launch_bounds__(256) void k_energy(const int* __restrict__ dims,
                                                const int* __restrict__ off,
                                                const float4* __restrict__ xyzs,
                                                const float* __restrict__ eatom, int n_models,
                                                long mstride, const double* __restrict__ eself,
                                                double* __restrict__ E, uint32_t* __restrict__ status) {
  __shared__ double part[4];
  __shared__ double es[kMaxS];  // self energies: no dependent global gather per atom
  const int n = dims[0], nmol = dims[1];
  const int m = blockIdx.x;
  if (m >= nmol) return;
  if (threadIdx.x < kMaxS) es[threadIdx.x] = eself[threadIdx.x];
  __syncthreads();
  int a = off[m], b = off[m + 1];
  a = a < 0 ? 0 : (a > n ? n : a);
  b = b < a ? a : (b > n ? n : b);
  double acc = 0.0;
  if (n_models == 1) {  // straight-line loop body: loads of several atoms in flight
#pragma unroll 4
    for (int i = a + (int)threadIdx.x; i < b; i += 256)
      acc += (double)eatom[i] + es[__float_as_int(xyzs[i].w) & (kMaxS - 1)];
  } else {
    const double inv_m = 1.0 / n_models;
    for (int i = a + (int)threadIdx.x; i < b; i += 256) {
      double e = (double)eatom[i];
      for (int k = 1; k < n_models; ++k) e += (double)eatom[k * mstride + i];
      acc += e * inv_m + es[__float_as_int(xyzs[i].w) & (kMaxS - 1)];
    }
  }
  acc = wave_sum_d(acc);
  if (lane_id() == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double e = ((part[0] + part[1]) + part[2]) + part[3];
    E[m] = e;
    if (!isfinite(e)) atomicOr(status, kStNonFinite);
  }
}

__global__ void k_fill_i32(int* __restrict__ p, int v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* __restrict__ p, float v, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ----------------------------------------------------------------- launchers

void launch_stage(int n_arg, int nmol_arg, int n_cap, int* dims, const float* pos,
                  const double* pos64, const int* gidx, int n_total, const int* species,
                  const int* off, int S, float4* xyzs, int* mol, float* Fzero, int* hist,
                  uint32_t* status, hipStream_t st) {
  const int nblk = stage_blocks(n_cap);
  hipLaunchKernelGGL(k_stage, dim3(nblk), dim3(256), 0, st, n_arg, nmol_arg, dims, pos, pos64,
                     gidx, n_total, species, off, S, xyzs, mol, Fzero, hist, status);
}

void launch_groups(const int* dims, int n_cap, int S, int* hist, GroupTable* gt, int* perm,
                   int rows_cap, const int* off, int wchunk_rows, uint32_t* status,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_groups, dim3(1), dim3(64 * kMaxS), 0, st, dims, stage_blocks(n_cap), S, hist, gt,
                     perm, rows_cap, off, wchunk_rows, status);
}

void launch_sort_scatter(const int* dims, int n_cap, int S, const float4* xyzs, const int* hist,
                         GroupTable* gt, int* row, int* perm, int rows_cap, const int* off,
                         int wchunk_rows, uint32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_sort_scatter, dim3(stage_blocks(n_cap)), dim3(256), 0, st, dims, S, xyzs,
                     hist, gt, row, perm, rows_cap, off, wchunk_rows, status);
}

void launch_scatter(const int* dims, int n_cap, int S, const float4* xyzs, const int* hist,
                    int* row, int* perm, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter, dim3(stage_blocks(n_cap)), dim3(256), 0, st, dims, S, xyzs, hist,
                     row, perm);
}

void launch_energy(const int* dims, int nmol_cap, const int* off, const float4* xyzs,
                   const float* eatom, int n_models, long mstride, const double* eself,
                   double* E, uint32_t* status, hipStream_t st) {
  if (nmol_cap <= 0) return;
  hipLaunchKernelGGL(k_energy, dim3(nmol_cap), dim3(256), 0, st, dims, off, xyzs, eatom,
                     n_models, mstride, eself, E, status);
}

void launch_fill_i32(int* p, int v, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
}

void launch_fill_f32(float* p, float v, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, v, n);
}

void launch_fill_f64(double* p, double v, int n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
}

}  // namespace nnp

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
#include "sort_scatter.h"
#include "energy_sum.h"

namespace nnp {

__global__ __launch_bounds__(256) void k_stage(int n_arg, int nmol_arg, int clear_status,
                                               int* __restrict__ dims,
                                               const float* __restrict__ pos,
                                               const double* __restrict__ pos64,
                                               const int* __restrict__ gidx, int n_total,
                                               const int* __restrict__ species,
                                               const int* __restrict__ off, int S,
                                               float4* __restrict__ xyzs, int* __restrict__ mol,
                                               int2* __restrict__ mrange,
                                               float* __restrict__ Fzero, int* __restrict__ hist,
                                               uint32_t* __restrict__ status,
                                               int* __restrict__ zero, int nzero) {
  __shared__ int h[kMaxS];
  // counters a later kernel of the evaluation accumulates into (the cell list)
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nzero; k += gridDim.x * blockDim.x)
    zero[k] = 0;
  __shared__ uint32_t bits;
  __shared__ int smp[kOffSamples + 1];
  const int n = n_arg >= 0 ? n_arg : dims[0];
  const int nmol = nmol_arg >= 0 ? nmol_arg : dims[1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (n_arg >= 0) {
      dims[0] = n;
      dims[1] = nmol;
    }
    // later kernels only add bits; an MD segment clears the word once, so
    // its bits accumulate over the steps
    if (clear_status) *status = 0u;
  }
  if (threadIdx.x < kMaxS) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) bits = 0;
  // every step-th molecule offset, step chosen so that at most kOffSamples
  // intervals remain: the molecule search runs in LDS and ends with at most
  // log2(step) dependent global loads (none for up to kOffSamples molecules)
  const int step = nmol > 0 ? (nmol + kOffSamples - 1) / kOffSamples : 1;
  const int K = nmol > 0 ? (nmol + step - 1) / step : 0;
  for (int k = threadIdx.x; k <= K; k += blockDim.x) {
    const int m = k * step;
    smp[k] = off[m < nmol ? m : nmol];
  }
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
    // molecule: the last m with off[m] <= i (off is non-decreasing when
    // valid), first over the samples, then inside one sample interval
    int klo = 0, khi = K;
    while (khi - klo > 1) {
      const int mid = (klo + khi) >> 1;
      if (smp[mid] <= i) klo = mid; else khi = mid;
    }
    int lo = klo * step, hi = khi * step < nmol ? khi * step : nmol;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid; else hi = mid;
    }
    mol[i] = lo;
    if (mrange) {  // the molecule's atom range, clamped to [0, n]
      int a = step == 1 ? smp[lo] : off[lo];
      int b = step == 1 ? smp[lo + 1 <= K ? lo + 1 : K] : off[lo + 1 <= nmol ? lo + 1 : nmol];
      a = a < 0 ? 0 : (a > n ? n : a);
      b = b < a ? a : (b > n ? n : b);
      mrange[i] = make_int2(a, b);
    }
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
// reduction, and the staging bits of the evaluation's status word (cleared
// by staging; every later kernel only adds bits).
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
  if (t == 0 && bits_all) atomicOr(status, bits_all);
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
// staging blocks.
__global__ __launch_bounds__(256) void k_sort_scatter(const int* __restrict__ dims, int S,
                                                      const float4* __restrict__ xyzs,
                                                      const int* __restrict__ hist,
                                                      GroupTable* __restrict__ gt,
                                                      int* __restrict__ row, int* __restrict__ perm,
                                                      int rows_cap, const int* __restrict__ off,
                                                      int wchunk_rows, uint32_t* __restrict__ status) {
  sort_scatter_block(blockIdx.x, gridDim.x, dims, S, xyzs, hist, gt, row, perm, rows_cap, off,
                     wchunk_rows, status);
}

__global__ __launch_bounds__(256) void k_energy(const int* __restrict__ dims, EnergyArgs A) {
  energy_block(blockIdx.x, dims, A);
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
                  const int* off, int S, float4* xyzs, int* mol, int2* mrange, float* Fzero,
                  int* hist, uint32_t* status, bool clear_status, int* zero, int nzero,
                  hipStream_t st) {
  const int nblk = stage_blocks(n_cap);
  hipLaunchKernelGGL(k_stage, dim3(nblk), dim3(256), 0, st, n_arg, nmol_arg, clear_status ? 1 : 0,
                     dims, pos, pos64, gidx, n_total, species, off, S, xyzs, mol, mrange, Fzero,
                     hist, status, zero, nzero);
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
  const EnergyArgs A{off, xyzs, eatom, n_models, mstride, eself, E, status};
  hipLaunchKernelGGL(k_energy, dim3(nmol_cap), dim3(256), 0, st, dims, A);
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

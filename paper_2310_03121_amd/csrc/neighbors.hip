// Neighbor search (one wavefront per atom).
//
// The paper lists neighbor-list construction among the operations its
// optimized kernels accelerate (Methods, "Optimization Through NNPOps").  The
// predicate is the float32 one documented in nnp.h (no FMA contraction,
// strict <), so the pair sets are reproducible bit for bit.
//
// Each wave scans candidates 64 at a time, evaluates the predicate per lane and
// compacts hits with a ballot and a prefix popcount into a per-wave LDS list of
// keys (angular flag, species, atom index).  The list is then ordered by key
// (angular neighbors first, grouped by species, ascending index) so that every
// later sum runs in a fixed order, and written to a fixed-capacity row
// (ELL layout: row i at i * cap) with counts (radial, angular), together
// with each neighbor's displacement and species, so that the symmetry
// function kernels start from the records instead of gathering positions.
//
// Molecules without a box: candidates are the atoms of the same molecule,
// read as contiguous float4 records.  Periodic boxes (one system): atoms are
// binned into cells no narrower than rc + 1e-3 A; a wave scans the
// concatenation of the 27 surrounding cells (fewer when a dimension has fewer
// than three cells) from a cell-ordered copy of the records.
#include "kernels.h"
#include "sort_scatter.h"

namespace nnp {

constexpr int kKeyJBits = 27;
constexpr int kKeyJMask = (1 << kKeyJBits) - 1;

__device__ __forceinline__ int make_key(int j, int s, bool ang) {
  return (ang ? 0 : (1 << 30)) | (s << kKeyJBits) | j;
}

// Sorts the wave's keys [0, nr) by rank (keys are distinct) and writes the
// row: indices to nbr, the matching displacement records to rec.
__device__ __forceinline__ void finish_list(const int* key, const float4* lrec, int nr, int na,
                                            int i, int cap, int* __restrict__ nbr,
                                            float4* __restrict__ rec, int2* __restrict__ counts) {
  const int lane = lane_id();
  for (int e = lane; e < nr; e += kWave) {
    const int k = key[e];
    int rank = 0;
    for (int q = 0; q < nr; ++q) rank += key[q] < k;
    nbr[(size_t)i * cap + rank] = k & kKeyJMask;
    rec[(size_t)i * cap + rank] = lrec[e];
  }
  if (lane == 0) counts[i] = make_int2(nr, na);
}

// Wave w of a block scans for atom i: the candidates are the atoms of its
// molecule, [mrange[i].x, mrange[i].y), read as contiguous records.
__device__ __forceinline__ void pairs_mol_wave(int i, int w, float4* lds, const AevConst& C,
                                               const float4* __restrict__ xyzs,
                                               const int2* __restrict__ mrange, int cap,
                                               int* __restrict__ nbr, float4* __restrict__ rec,
                                               int2* __restrict__ counts,
                                               uint32_t* __restrict__ status) {
  const int lane = lane_id();
  float4* lrec = lds + (size_t)w * cap;
  int* key = reinterpret_cast<int*>(lds + (size_t)4 * cap) + w * cap;
  const float4 pi = xyzs[i];
  const int2 ab = mrange[i];  // clamped to [0, n] by staging
  const int a = ab.x, b = ab.y;
  int nr = 0, na = 0;
  for (int base = a; base < b; base += kWave) {
    const int j = base + lane;
    bool inR = false, inA = false;
    int sj = 0;
    float dx = 0.f, dy = 0.f, dz = 0.f;
    if (j < b && j != i) {
      const float4 pj = xyzs[j];
      dx = __fsub_rn(pj.x, pi.x);
      dy = __fsub_rn(pj.y, pi.y);
      dz = __fsub_rn(pj.z, pi.z);
      const float d2 = dist2(dx, dy, dz);
      inR = d2 < C.rc2_r;
      inA = d2 < C.rc2_a;
      sj = species_of(pj);
    }
    const uint64_t mr = ballot(inR);
    const int p = nr + popc_below(mr);
    if (inR && p < cap) {
      key[p] = make_key(j, sj, inA);
      lrec[p] = make_float4(dx, dy, dz, __int_as_float(sj));
    }
    nr += __popcll(mr);
    na += __popcll(ballot(inA));
  }
  if (nr > cap) {
    if (lane == 0) atomicOr(status, kStCapacity);
    nr = cap;
    na = na < nr ? na : nr;
  }
  wave_lds_sync();
  finish_list(key, lrec, nr, na, i, cap, nbr, rec, counts);
}

__global__ __launch_bounds__(256) void k_pairs_mol(const int* __restrict__ dims, AevConst C,
                                                   const float4* __restrict__ xyzs,
                                                   const int2* __restrict__ mrange, int cap,
                                                   int* __restrict__ nbr, float4* __restrict__ rec,
                                                   int2* __restrict__ counts,
                                                   uint32_t* __restrict__ status) {
  extern __shared__ float4 lds_mol[];
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  if (i >= dims[0]) return;
  pairs_mol_wave(i, w, lds_mol, C, xyzs, mrange, cap, nbr, rec, counts, status);
}

// The species sort (blocks [0, nsort)) and the molecule neighbor search (the
// blocks after them) in one launch: both read only what staging wrote, and
// the pair scan no longer waits behind the sort's tail.
__global__ __launch_bounds__(256) void k_sort_pairs_mol(
    const int* __restrict__ dims, int nsort, int S, const int* __restrict__ hist,
    GroupTable* __restrict__ gt, int* __restrict__ row, int* __restrict__ perm, int rows_cap,
    const int* __restrict__ off, int wchunk_rows, AevConst C, const float4* __restrict__ xyzs,
    const int2* __restrict__ mrange, int cap, int* __restrict__ nbr, float4* __restrict__ rec,
    int2* __restrict__ counts, uint32_t* __restrict__ status) {
  extern __shared__ float4 lds_mol[];
  if ((int)blockIdx.x < nsort) {  // block-uniform
    sort_scatter_block(blockIdx.x, nsort, dims, S, xyzs, hist, gt, row, perm, rows_cap, off,
                       wchunk_rows, status);
    return;
  }
  const int w = threadIdx.x >> 6;
  const int i = ((int)blockIdx.x - nsort) * 4 + w;
  if (i >= dims[0]) return;
  pairs_mol_wave(i, w, lds_mol, C, xyzs, mrange, cap, nbr, rec, counts, status);
}

// ---------------------------------------------------------------- cell list

__device__ __forceinline__ int cell_coord(float x, float L, float invL, float scale, int nc) {
  // wrap into [0, L) then bin; clamped so that rounding and bad input stay in range
  float xw = x - L * floorf(x * invL);
  int c = (int)(xw * scale);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ __launch_bounds__(256) void k_cell_count(const int* __restrict__ dims, BoxConst B,
                                                    const float4* __restrict__ xyzs,
                                                    int* __restrict__ cell_of,
                                                    int* __restrict__ cell_cnt) {
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 p = xyzs[i];
  int cx, cy, cz;
  if (B.periodic == 2) {
    // fractional coordinates, wrapped into [0, 1), then binned
    const float sz = p.z * B.inv_diag[2];
    const float sy = (p.y - B.v[2][1] * sz) * B.inv_diag[1];
    const float sx = (p.x - B.v[1][0] * sy - B.v[2][0] * sz) * B.inv_diag[0];
    cx = cell_coord(sx, 1.f, 1.f, (float)B.nc[0], B.nc[0]);
    cy = cell_coord(sy, 1.f, 1.f, (float)B.nc[1], B.nc[1]);
    cz = cell_coord(sz, 1.f, 1.f, (float)B.nc[2], B.nc[2]);
  } else {
    cx = cell_coord(p.x, B.L[0], B.invL[0], B.cell_scale[0], B.nc[0]);
    cy = cell_coord(p.y, B.L[1], B.invL[1], B.cell_scale[1], B.nc[1]);
    cz = cell_coord(p.z, B.L[2], B.invL[2], B.cell_scale[2], B.nc[2]);
  }
  const int c = cx + B.nc[0] * (cy + B.nc[1] * cz);
  cell_of[i] = c;
  atomicAdd(&cell_cnt[c], 1);
}

// One block: exclusive scan of the cell counts into starts and cursors.
__global__ __launch_bounds__(1024) void k_cell_scan(int ncell, const int* __restrict__ cnt,
                                                    int* __restrict__ start,
                                                    int* __restrict__ cursor) {
  __shared__ int scan[1024];
  const int t = threadIdx.x;
  int carry = 0;
  for (int c0 = 0; c0 < ncell; c0 += blockDim.x) {
    const int c = c0 + t;
    const int v = c < ncell ? cnt[c] : 0;
    scan[t] = v;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      int u = t >= o ? scan[t - o] : 0;
      __syncthreads();
      scan[t] += u;
      __syncthreads();
    }
    if (c < ncell) {
      start[c] = carry + scan[t] - v;
      cursor[c] = carry + scan[t] - v;
    }
    const int last = scan[blockDim.x - 1];
    __syncthreads();
    carry += last;
  }
  if (t == 0) start[ncell] = carry;
}

__global__ __launch_bounds__(256) void k_cell_fill(const int* __restrict__ dims,
                                                   const float4* __restrict__ xyzs,
                                                   const int* __restrict__ cell_of,
                                                   int* __restrict__ cursor,
                                                   int* __restrict__ cell_atoms,
                                                   float4* __restrict__ cell_xyzs) {
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int slot = atomicAdd(&cursor[cell_of[i]], 1);
  cell_atoms[slot] = i;
  cell_xyzs[slot] = xyzs[i];
}

// One wave per atom, visiting atoms in cell order (neighbouring waves share
// their candidate cells).  Candidates are the concatenation of the stencil
// cells; a lane maps its candidate number to (cell, slot) through a per-wave
// prefix table of the stencil's cell sizes.
__global__ __launch_bounds__(256) void k_pairs_cell(const int* __restrict__ dims, AevConst C,
                                                    BoxConst B, const int* __restrict__ cell_of,
                                                    const int* __restrict__ cell_start,
                                                    const int* __restrict__ cell_atoms,
                                                    const float4* __restrict__ cell_xyzs, int cap,
                                                    int* __restrict__ nbr,
                                                    float4* __restrict__ rec,
                                                    int2* __restrict__ counts,
                                                    uint32_t* __restrict__ status) {
  extern __shared__ float4 lds_cell[];
  const int n = dims[0];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int slot_i = blockIdx.x * 4 + w;
  if (slot_i >= n) return;
  float4* lrec = lds_cell + (size_t)w * cap;
  int* key = reinterpret_cast<int*>(lds_cell + (size_t)4 * cap) + w * (cap + 64);
  int* pref = key + cap;  // 28 prefix entries + 27 cell starts
  int* cst = pref + 28;
  const int i = cell_atoms[slot_i];
  const float4 pi = cell_xyzs[slot_i];
  const int c = cell_of[i];
  const int cx = c % B.nc[0], cy = (c / B.nc[0]) % B.nc[1], cz = c / (B.nc[0] * B.nc[1]);
  // stencil: offsets -1..1 per binned dimension, only 0 where nc == 1
  const int rx = B.nc[0] >= 3 ? 1 : 0, ry = B.nc[1] >= 3 ? 1 : 0, rz = B.nc[2] >= 3 ? 1 : 0;
  const int sx = 2 * rx + 1, sy = 2 * ry + 1, sz = 2 * rz + 1;
  const int nst = sx * sy * sz;
  int cnt = 0, st = 0;
  if (lane < nst) {
    const int ox = lane % sx - rx, oy = (lane / sx) % sy - ry, oz = lane / (sx * sy) - rz;
    const int ncx = (cx + ox + B.nc[0]) % B.nc[0];
    const int ncy = (cy + oy + B.nc[1]) % B.nc[1];
    const int ncz = (cz + oz + B.nc[2]) % B.nc[2];
    const int cc = ncx + B.nc[0] * (ncy + B.nc[1] * ncz);
    st = cell_start[cc];
    cnt = cell_start[cc + 1] - st;
  }
  // inclusive scan of cnt over lanes 0..nst-1
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane < nst) {
    pref[lane + 1] = incl;
    cst[lane] = st;
  }
  if (lane == 0) pref[0] = 0;
  const int total = __shfl(incl, nst - 1, 64);
  wave_lds_sync();
  int nr = 0, na = 0;
  for (int base = 0; base < total; base += kWave) {
    const int t = base + lane;
    bool inR = false, inA = false;
    int j = 0, sj = 0;
    float dx = 0.f, dy = 0.f, dz = 0.f;
    if (t < total) {
      // largest q < nst with pref[q] <= t (that cell is non-empty and holds t)
      int q = 0, hi = nst;
      while (hi - q > 1) {
        const int mid = (q + hi) >> 1;
        if (pref[mid] <= t) q = mid; else hi = mid;
      }
      const int slot = cst[q] + (t - pref[q]);
      j = cell_atoms[slot];
      if (j != i) {
        const float4 pj = cell_xyzs[slot];
        if (B.periodic == 2) {
          tric_disp(pi, pj, B, dx, dy, dz);
        } else {
          dx = disp(pi.x, pj.x, B.L[0], B.invL[0], 1);
          dy = disp(pi.y, pj.y, B.L[1], B.invL[1], 1);
          dz = disp(pi.z, pj.z, B.L[2], B.invL[2], 1);
        }
        const float d2 = dist2(dx, dy, dz);
        inR = d2 < C.rc2_r;
        inA = d2 < C.rc2_a;
        sj = species_of(pj);
      }
    }
    const uint64_t mr = ballot(inR);
    const int p = nr + popc_below(mr);
    if (inR && p < cap) {
      key[p] = make_key(j, sj, inA);
      lrec[p] = make_float4(dx, dy, dz, __int_as_float(sj));
    }
    nr += __popcll(mr);
    na += __popcll(ballot(inA));
  }
  if (nr > cap) {
    if (lane == 0) atomicOr(status, kStCapacity);
    nr = cap;
    na = na < nr ? na : nr;
  }
  wave_lds_sync();
  finish_list(key, lrec, nr, na, i, cap, nbr, rec, counts);
}

// ----------------------------------------------------------------- launchers

void launch_pairs_mol(const int* dims, int n_cap, const AevConst& C, const float4* xyzs,
                      const int2* mrange, int cap, int* nbr, float4* rec, int2* counts,
                      uint32_t* status, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_pairs_mol, dim3((n_cap + 3) / 4), dim3(256),
                     4 * cap * (sizeof(float4) + sizeof(int)), st, dims, C, xyzs, mrange, cap, nbr,
                     rec, counts, status);
}

void launch_sort_pairs_mol(const int* dims, int n_cap, int S, const int* hist, GroupTable* gt,
                           int* row, int* perm, int rows_cap, const int* off, int wchunk_rows,
                           const AevConst& C, const float4* xyzs, const int2* mrange, int cap,
                           int* nbr, float4* rec, int2* counts, uint32_t* status,
                           hipStream_t st) {
  const int nsort = stage_blocks(n_cap);
  const int npair = n_cap > 0 ? (n_cap + 3) / 4 : 0;
  hipLaunchKernelGGL(k_sort_pairs_mol, dim3(nsort + npair), dim3(256),
                     4 * cap * (sizeof(float4) + sizeof(int)), st, dims, nsort, S, hist, gt, row,
                     perm, rows_cap, off, wchunk_rows, C, xyzs, mrange, cap, nbr, rec, counts,
                     status);
}

void launch_pairs_cell(const int* dims, int n_cap, const AevConst& C, const BoxConst& B,
                       const float4* xyzs, int* cell_of, int* cell_cnt, int* cell_start,
                       int* cursor, int* cell_atoms, float4* cell_xyzs, int cap, int* nbr,
                       float4* rec, int2* counts, uint32_t* status, hipStream_t st) {
  if (n_cap <= 0) return;
  const int ncell = B.nc[0] * B.nc[1] * B.nc[2];
  hipLaunchKernelGGL(k_fill_i32, dim3((ncell + 255) / 256), dim3(256), 0, st, cell_cnt, 0, ncell);
  hipLaunchKernelGGL(k_cell_count, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, B, xyzs,
                     cell_of, cell_cnt);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, st, ncell, cell_cnt, cell_start,
                     cursor);
  hipLaunchKernelGGL(k_cell_fill, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, xyzs,
                     cell_of, cursor, cell_atoms, cell_xyzs);
  hipLaunchKernelGGL(k_pairs_cell, dim3((n_cap + 3) / 4), dim3(256),
                     4 * (cap * sizeof(float4) + (cap + 64) * sizeof(int)), st, dims, C, B,
                     cell_of, cell_start, cell_atoms, cell_xyzs, cap, nbr, rec, counts, status);
}

}  // namespace nnp

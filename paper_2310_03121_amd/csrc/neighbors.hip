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
// binned into cells no narrower than rc + 1e-3 A; a workgroup per cell stages
// the concatenation of the 27 surrounding cells (fewer when a dimension has
// fewer than three cells) in LDS from a cell-ordered copy of the records, and
// its waves scan it for the cell's atoms.
#include "kernels.h"
#include "sort_scatter.h"

namespace nnp {

constexpr int kKeyJBits = 27;
constexpr int kKeyJMask = (1 << kKeyJBits) - 1;

__device__ __forceinline__ int make_key(int j, int s, bool ang) {
  return (ang ? 0 : (1 << 30)) | (s << kKeyJBits) | j;
}

// Sorts the wave's keys [0, nr) by rank (keys are distinct) and writes the
// row: indices to nbr, the matching displacement records to rec.  Lists of at
// most 64 keep one key per lane and count smaller keys with lane reads (no
// LDS round trip per comparison), in groups of 16 up to nr; longer lists
// compare against the LDS copy.
__device__ __forceinline__ void finish_list(const int* key, const float4* lrec, int nr, int na,
                                            int i, int cap, int* __restrict__ nbr,
                                            float4* __restrict__ rec, int2* __restrict__ counts) {
  const int lane = lane_id();
  if (nr <= kWave) {
    const int k = lane < nr ? key[lane] : 0x7fffffff;
    int rank = 0;
    for (int g = 0; g < nr; g += 16) {
#pragma unroll
      for (int q = 0; q < 16; ++q) rank += __builtin_amdgcn_readlane(k, g + q) < k ? 1 : 0;
    }
    if (lane < nr) {
      nbr[(size_t)i * cap + rank] = k & kKeyJMask;
      rec[(size_t)i * cap + rank] = lrec[lane];
    }
  } else {
    for (int e = lane; e < nr; e += kWave) {
      const int k = key[e];
      int rank = 0;
      for (int q = 0; q < nr; ++q) rank += key[q] < k;
      nbr[(size_t)i * cap + rank] = k & kKeyJMask;
      rec[(size_t)i * cap + rank] = lrec[e];
    }
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

// Bins the atoms (cell counts by atomics; staging zeroed the counts and the
// done counter cell_cnt[ncell]), and the last workgroup to finish turns the
// counts into cell starts and fill cursors (an exclusive scan), so binning
// needs no launch of its own for the scan.  Every workgroup takes part in the
// done count, whatever its atoms.
// Scan: the workgroup that finishes last also turns the counts into cell
// starts (boxes with more cells than k_cell_fill_scan's LDS holds).
template <bool Scan>
__global__ __launch_bounds__(256) void k_cell_count(const int* __restrict__ dims, BoxConst B,
                                                    const float4* __restrict__ xyzs,
                                                    int* __restrict__ cell_of,
                                                    int* __restrict__ cell_cnt, int ncell,
                                                    int* __restrict__ start,
                                                    int* __restrict__ cursor) {
  __shared__ int scan[256];
  __shared__ int is_last;
  const int n = dims[0];
  const int t = threadIdx.x;
  const int i = blockIdx.x * blockDim.x + t;
  if (i < n) {
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
  if constexpr (!Scan) return;
  __threadfence();
  __syncthreads();
  if (t == 0) is_last = atomicAdd(&cell_cnt[ncell], 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  // Exclusive scan of the counts, 2,048 cells per pass: each thread loads its
  // eight consecutive counts at once (one memory latency per pass, not one per
  // 256 cells), scans their sums across the block and writes eight starts.
  constexpr int kPer = 8;
  int carry = 0;
  for (int c0 = 0; c0 < ncell; c0 += 256 * kPer) {
    const int cb = c0 + t * kPer;
    int v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      v[q] = cb + q < ncell ? __hip_atomic_load(&cell_cnt[cb + q], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                            : 0;
    int sum = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) sum += v[q];
    scan[t] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      const int u = t >= o ? scan[t - o] : 0;
      __syncthreads();
      scan[t] += u;
      __syncthreads();
    }
    int run = carry + scan[t] - sum;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (cb + q < ncell) {
        start[cb + q] = run;
        cursor[cb + q] = run;
      }
      run += v[q];
    }
    const int last = scan[255];
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

// Up to kCellScanLds cells: every workgroup scans the cell counts into LDS
// itself (they are few: one pass of loads, no done counter and no
// single-workgroup tail), workgroup 0 writes the starts for the pair search,
// and each atom takes its slot from a per-cell fill counter.
__global__ __launch_bounds__(256) void k_cell_fill_scan(
    const int* __restrict__ dims, const float4* __restrict__ xyzs,
    const int* __restrict__ cell_of, const int* __restrict__ cnt, int* __restrict__ fillc,
    int ncell, int* __restrict__ start_out, int* __restrict__ cell_atoms,
    float4* __restrict__ cell_xyzs) {
  __shared__ int st[kCellScanLds + 1];
  __shared__ int scan[256];
  const int t = threadIdx.x;
  constexpr int kPer = kCellScanLds / 256;
  const int cb = t * kPer;
  int v[kPer];
  int sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = cb + q < ncell ? cnt[cb + q] : 0;
    sum += v[q];
  }
  scan[t] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int u = t >= o ? scan[t - o] : 0;
    __syncthreads();
    scan[t] += u;
    __syncthreads();
  }
  int run = scan[t] - sum;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (cb + q < ncell) st[cb + q] = run;
    run += v[q];
  }
  if (t == 255) st[ncell < kCellScanLds ? ncell : kCellScanLds] = scan[255];
  __syncthreads();
  if (blockIdx.x == 0)
    for (int c = t; c <= ncell; c += 256) start_out[c] = st[c];
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + t;
  if (i >= n) return;
  const int c = cell_of[i];
  const int slot = st[c] + atomicAdd(&fillc[c], 1);
  cell_atoms[slot] = i;
  cell_xyzs[slot] = xyzs[i];
}

// Cell-centred neighbor search: one workgroup per cell.  The workgroup stages
// the records and indices of its stencil cells (the concatenation of up to 27
// cells, at most kCandLds of them) in LDS once; its waves then take the
// cell's atoms in turn and scan the staged candidates 64 at a time, so the
// ~460 candidates of a liquid-density cell are read from global memory once
// per cell instead of once per atom.  A workgroup whose stencil holds more
// candidates reads them from global memory (the same arithmetic).
constexpr int kCandLds = 1024;

// Waves per cell workgroup: about two atoms each at liquid density (17 per
// cell in the large box).  Measured there: 16 waves 55.8 us (most waves take
// one atom, and the workgroup holds its LDS until its slowest wave ends),
// 8 waves 47.4 us, 4 waves 58.9 us.
__host__ __device__ constexpr int pairs_cell_waves(int cap) {
  return cap <= 128 ? 8 : 4;
}

__host__ __device__ constexpr size_t pairs_cell_lds_bytes(int cap) {
  return (size_t)kCandLds * (sizeof(float4) + sizeof(int)) +
         (size_t)pairs_cell_waves(cap) * cap * (sizeof(float4) + sizeof(int)) + 64 * sizeof(int);
}

__global__ __launch_bounds__(1024) void k_pairs_cell_lds(
    const int* __restrict__ dims, AevConst C, BoxConst B, const int* __restrict__ cell_start,
    const int* __restrict__ cell_atoms, const float4* __restrict__ cell_xyzs, int cap,
    int* __restrict__ nbr, float4* __restrict__ rec, int2* __restrict__ counts,
    uint32_t* __restrict__ status, int splits) {
  extern __shared__ float4 lds_cell[];
  float4* cand = lds_cell;
  int* cidx = reinterpret_cast<int*>(cand + kCandLds);
  const int nw = (int)blockDim.x >> 6;
  float4* lrec_all = reinterpret_cast<float4*>(cidx + kCandLds);
  int* key_all = reinterpret_cast<int*>(lrec_all + (size_t)nw * cap);
  int* pref = key_all + (size_t)nw * cap;  // 28 prefix entries
  int* cst = pref + 28;                   // 27 cell starts
  const int n = dims[0];
  const int tid = threadIdx.x, lane = lane_id();
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  float4* lrec = lrec_all + (size_t)w * cap;
  int* key = key_all + (size_t)w * cap;
  // workgroups (c, part): with few cells, `splits` workgroups share a cell's
  // atoms (each stages the cell's candidates)
  const int c = (int)blockIdx.x / splits, part = (int)blockIdx.x % splits;
  const int cx = c % B.nc[0], cy = (c / B.nc[0]) % B.nc[1], cz = c / (B.nc[0] * B.nc[1]);
  // stencil: offsets -1..1 per binned dimension, only 0 where nc == 1
  const int rx = B.nc[0] >= 3 ? 1 : 0, ry = B.nc[1] >= 3 ? 1 : 0, rz = B.nc[2] >= 3 ? 1 : 0;
  const int sx = 2 * rx + 1, sy = 2 * ry + 1, sz = 2 * rz + 1;
  const int nst = sx * sy * sz;
  if (w == 0) {
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
  }
  __syncthreads();
  const int total = pref[nst];
  const bool staged = total <= kCandLds;  // block-uniform
  // slot of candidate t: the largest q < nst with pref[q] <= t holds it
  auto cand_slot = [&](int t) __attribute__((always_inline)) {
    int q = 0, hi = nst;
    while (hi - q > 1) {
      const int mid = (q + hi) >> 1;
      if (pref[mid] <= t) q = mid; else hi = mid;
    }
    return cst[q] + (t - pref[q]);
  };
  if (staged) {
    for (int t = tid; t < total; t += (int)blockDim.x) {
      const int slot = cand_slot(t);
      cand[t] = cell_xyzs[slot];
      cidx[t] = cell_atoms[slot];
    }
  }
  __syncthreads();
  const int c0 = cell_start[c], cn = cell_start[c + 1] - c0;
  for (int a = part * nw + w; a < cn; a += nw * splits) {
    const int i = cell_atoms[c0 + a];
    const float4 pi = cell_xyzs[c0 + a];
    int nr = 0, na = 0;
    for (int base = 0; base < total; base += kWave) {
      const int t = base + lane;
      bool inR = false, inA = false;
      int j = 0, sj = 0;
      float dx = 0.f, dy = 0.f, dz = 0.f;
      if (t < total) {
        float4 pj;
        if (staged) {
          j = cidx[t];
          pj = cand[t];
        } else {
          const int slot = cand_slot(t);
          j = cell_atoms[slot];
          pj = cell_xyzs[slot];
        }
        if (j != i) {
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
    if (i >= 0 && i < n) finish_list(key, lrec, nr, na, i, cap, nbr, rec, counts);
    wave_lds_sync();  // the next atom reuses the wave's list
  }
}

// ------------------------------------------------------------ force gather

// Sort key of entry q of atom j's list (the key its row was ordered by).
__device__ __forceinline__ int entry_key(const int* __restrict__ nbr,
                                         const float4* __restrict__ rec, int j, int q, int na,
                                         int cap) {
  const size_t o = (size_t)j * cap + q;
  return make_key(nbr[o] & kKeyJMask, species_of(rec[o]), q < na);
}

__global__ __launch_bounds__(256) void k_force_gather(
    const int* __restrict__ dims, const float4* __restrict__ xyzs, const float4* __restrict__ rec,
    const int* __restrict__ nbr, const int2* __restrict__ counts, int cap,
    const float4* __restrict__ pgrad, float* __restrict__ out, float sign,
    const int* __restrict__ gidx, int n_total) {
  const int n = dims[0];
  const int a = (int)blockIdx.x * 4 + ((int)threadIdx.x >> 6);
  if (a >= n) return;
  const int lane = lane_id();
  const int2 ca = counts[a];
  const int nr = ca.x < 0 ? 0 : (ca.x > cap ? cap : ca.x);
  const int na = ca.y < 0 ? 0 : (ca.y > nr ? nr : ca.y);
  const int sa = species_of(xyzs[a]);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int e = lane; e < nr; e += kWave) {
    const int j = clampi(nbr[(size_t)a * cap + e], n);
    // the same pair seen from j: same distance, so the same angular flag
    const int key = make_key(a, sa, e < na);
    const int2 cj = counts[j];
    const int nrj = cj.x < 0 ? 0 : (cj.x > cap ? cap : cj.x);
    const int naj = cj.y < 0 ? 0 : (cj.y > nrj ? nrj : cj.y);
    int lo = 0, hi = nrj;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (entry_key(nbr, rec, j, mid, naj, cap) < key) lo = mid + 1; else hi = mid;
    }
    const float4 own = pgrad[(size_t)a * cap + e];
    float4 oth = make_float4(0.f, 0.f, 0.f, 0.f);
    // (absent only when a list was cut at capacity, which the status reports)
    if (lo < nrj && entry_key(nbr, rec, j, lo, naj, cap) == key) oth = pgrad[(size_t)j * cap + lo];
    fx += own.x - oth.x;
    fy += own.y - oth.y;
    fz += own.z - oth.z;
  }
  fx = wave_sum_rows(fx);
  fy = wave_sum_rows(fy);
  fz = wave_sum_rows(fz);
  if (lane == 0) {
    int row = a;
    if (gidx) {
      row = gidx[a];
      if (row < 0 || row >= n_total) return;
    }
    // added, as the scatter adds (staging zeroed the rows of a whole-system
    // call; a subset call adds to the caller's rows, each written once)
    out[3 * (size_t)row] += sign * fx;
    out[3 * (size_t)row + 1] += sign * fy;
    out[3 * (size_t)row + 2] += sign * fz;
  }
}

void launch_force_gather(const int* dims, int n_cap, const float4* xyzs, const float4* rec,
                         const int* nbr, const int2* counts, int cap, const float4* pgrad,
                         float* out, float sign, const int* gidx, int n_total, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_force_gather, dim3((n_cap + 3) / 4), dim3(256), 0, st, dims, xyzs, rec,
                     nbr, counts, cap, pgrad, out, sign, gidx, n_total);
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
  // staging zeroed cell_cnt[0 .. cell_zero_ints(ncell))
  const dim3 grid((n_cap + 255) / 256);
  if (ncell <= kCellScanLds) {
    hipLaunchKernelGGL(k_cell_count<false>, grid, dim3(256), 0, st, dims, B, xyzs, cell_of,
                       cell_cnt, ncell, cell_start, cursor);
    hipLaunchKernelGGL(k_cell_fill_scan, grid, dim3(256), 0, st, dims, xyzs, cell_of, cell_cnt,
                       cell_cnt + ncell, ncell, cell_start, cell_atoms, cell_xyzs);
  } else {
    hipLaunchKernelGGL(k_cell_count<true>, grid, dim3(256), 0, st, dims, B, xyzs, cell_of,
                       cell_cnt, ncell, cell_start, cursor);
    hipLaunchKernelGGL(k_cell_fill, grid, dim3(256), 0, st, dims, xyzs, cell_of, cursor,
                       cell_atoms, cell_xyzs);
  }
  static const bool attr = (ensure_lds(k_pairs_cell_lds), true);
  (void)attr;
  // at least about four workgroups per CU: boxes with few cells split them
  const int splits = ncell >= 1024 ? 1 : (ncell >= 512 ? 2 : 4);
  hipLaunchKernelGGL(k_pairs_cell_lds, dim3(ncell * splits), dim3(64 * pairs_cell_waves(cap)),
                     pairs_cell_lds_bytes(cap), st, dims, C, B, cell_start, cell_atoms, cell_xyzs,
                     cap, nbr, rec, counts, status, splits);
}

}  // namespace nnp

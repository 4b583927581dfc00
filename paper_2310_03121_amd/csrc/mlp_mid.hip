// Fused middle of the per-element networks (BF16 operands, FP32 accumulate):
// layer 2, the energy head, and the adjoint of layers 3 and 2, for one tile of
// 128 species-sorted rows per workgroup.
//
//   H2 = CELU(H1 W1^T + b1)                       (kept in LDS)
//   z3 = H2 W2^T + b2;  E_i = w_out . CELU(z3) + b_out
//   D3 = up_i * w_out * CELU'(z3)                 (kept in LDS, over H1)
//   D2 = (D3 W2) * CELU'(z2)                      (written over H2 in LDS)
//   D1 = (D2 W1) * CELU'(z1)                      (to global)
//
// CELU'(z) is recovered from the stored activation: 1 for h > 0, else
// 1 + h/alpha (for D1 from H1 in global memory, which the tile loaded at the
// start and which is still L2 resident; it is fetched ahead of the last
// product).  Every global load is issued well ahead of its use: the tile's H1
// vectors all before their LDS stores, the first weights before the tile.  The four products are MFMA GEMMs
// with the A operand resident in LDS and the weights streamed into registers
// (mfma_tile.h); 8 waves per workgroup.  This removes three launches and the
// HBM round trips of H2, D3 and D2 that separate layer kernels would need.
// Optional pointers also store H2, H3, D3 and D2 for the parameter gradients.
#include "mfma_tile.h"

namespace nnp {

constexpr int kMidBM = 128;

// Wave layout of a product with N columns over a tile of BM rows in one
// pass: BM/64 x 4 waves of 64 x (N/4) when N is a multiple of 64, else
// BM/32 x 2 waves of 32 x (N/2) (eight waves for 128 rows, four for 64).
template <int N, int BM = kMidBM>
struct MidCfg {
  static constexpr bool wide = N % 64 == 0;
  static constexpr int WN = wide ? 4 : 2;
  static constexpr int TM = wide ? 4 : 2;
  static constexpr int WM = BM / (16 * TM);
  static constexpr int TN = wide ? N / 64 : N / 32;
  static constexpr int P = 4;  // weight ring depth (k-steps)
  static_assert(WM * TM * 16 == BM && WN * TN * 16 == N, "one pass covers N");
  static_assert(WM * WN * 64 == BM * 4, "the same waves for every product");
};

template <int N, int BM = kMidBM>
using MidRing = BRing<bf16_t, MidCfg<N, BM>::TN, MidCfg<N, BM>::P>;

// Starts the weight ring of a product with N columns and K inner (the
// weights do not depend on the activations, so this can run early).
template <int N, int K, int BM = kMidBM>
__device__ __forceinline__ void mid_ring(MidRing<N, BM>& br, const bf16_t* B, int lane, int wv) {
  static_assert(K % Frag<bf16_t>::KS == 0, "whole k-steps");
  br.init(B, (wv % MidCfg<N, BM>::WN) * MidCfg<N, BM>::TN * 16, -1, lane, K);
  br.prologue();
}

// acc = A (LDS, row stride sa bytes, K columns) * B^T, B from a started ring.
template <int N, int K, int BM = kMidBM>
__device__ __forceinline__ void mid_steps(const unsigned char* As, int sa, MidRing<N, BM>& br,
                                          int lane, int wv,
                                          f32x4_t (&acc)[MidCfg<N, BM>::TM][MidCfg<N, BM>::TN]) {
  using C = MidCfg<N, BM>;
  const int wm = wv / C::WN;
  zero_acc(acc);
  const unsigned char* a0 = As + (wm * C::TM * 16 + (lane & 15)) * sa + (lane >> 4) * 16;
  uint4 fe[C::TM], fo[C::TM];
  ksteps_ct<bf16_t, C::TM, C::TN, C::P, K / Frag<bf16_t>::KS>(a0, 16 * sa, br, acc, fe, fo);
}

__device__ __forceinline__ void lds_put4(unsigned char* p, float4 v) {
  *reinterpret_cast<uint2*>(p) = make_uint2(f2bf2(v.x, v.y), f2bf2(v.z, v.w));
}

__device__ __forceinline__ float4 lds_get4(const unsigned char* p) {
  const uint2 u = *reinterpret_cast<const uint2*>(p);
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
}

// The four products of the fused middle, from H1 in X1 (LDS, row stride S1)
// with the first product's weight ring already started: H2 into X2,
// energies, D3 into D3s (row stride S3; X1 itself when H1 need not stay),
// D2 over H2, and D1 to global a.D1 (if set) and to LDS d1_lds (if set, row
// stride S1, which may be X1: D3 is consumed by then).  The last product's
// slopes come from H1 in X1 when it is still there (D3s elsewhere), else
// from global a.H1.  after_last() runs right after the last product's steps
// (a following product can start its weight ring there).
template <int W1, int W2, int W3, int BM, typename AfterLast>
__device__ __forceinline__ void mid_products(const MidArgs& a, MidRing<W2, BM>& br1,
                                             unsigned char* X1, unsigned char* X2, float* epart,
                                             int row0, int row_end, int s,
                                             unsigned char* d1_lds, unsigned char* D3s, int S3,
                                             AfterLast&& after_last) {
  constexpr int S1 = W1 * 2 + 16, S2 = W2 * 2 + 16;
  (void)S2;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rl = lane & 15, cq = (lane >> 4) * 4;
  const float alpha = a.alpha, ia = 1.f / a.alpha, ial2e = a.inv_alpha_l2e;
  // (each product's weight ring starts right after the previous product's
  // last step, so its first fragments arrive during that epilogue and
  // barrier instead of after them)
  MidRing<W3, BM> br2;
  // ---- H2 = CELU(H1 W1^T + b1)
  {
    using C = MidCfg<W2, BM>;
    f32x4_t acc[C::TM][C::TN];
    mid_steps<W2, W1, BM>(X1, S1, br1, lane, wv, acc);
    mid_ring<W3, W2, BM>(br2, a.W2 + (size_t)s * W3 * W2, lane, wv);
    const int wm = wv / C::WN, wn = wv % C::WN;
    const float* b1 = a.b1 + (size_t)s * W2;
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int r = wm * C::TM * 16 + i * 16 + rl;
      const bool rv = row0 + r < row_end;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int c = wn * C::TN * 16 + j * 16 + cq;
        const float4 b = *reinterpret_cast<const float4*>(b1 + c);
        float4 h = make_float4(celu_fwd(acc[i][j][0] + b.x, alpha, ial2e),
                               celu_fwd(acc[i][j][1] + b.y, alpha, ial2e),
                               celu_fwd(acc[i][j][2] + b.z, alpha, ial2e),
                               celu_fwd(acc[i][j][3] + b.w, alpha, ial2e));
        if (!rv) h = make_float4(0.f, 0.f, 0.f, 0.f);
        lds_put4(X2 + r * S2 + c * 2, h);
        if (a.H2) Store<bf16_t>::put4(a.H2 + (size_t)(row0 + r) * W2 + c, h);
      }
    }
  }
  __syncthreads();

  // ---- z3 = H2 W2^T + b2: energies and D3 (over H1)
  MidRing<W2, BM> br3;
  {
    using C = MidCfg<W3, BM>;
    f32x4_t acc[C::TM][C::TN];
    mid_steps<W3, W2, BM>(X2, S2, br2, lane, wv, acc);
    mid_ring<W2, W3, BM>(br3, a.W2T + (size_t)s * W2 * W3, lane, wv);
    const int wm = wv / C::WN, wn = wv % C::WN;
    const float* b2 = a.b2 + (size_t)s * W3;
    const float* wo = a.wout + (size_t)s * W3;
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int r = wm * C::TM * 16 + i * 16 + rl;
      const int row = row0 + r;
      const bool rv = row < row_end;
      float up = 0.f;
      if (rv) up = (a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f) * a.escale;
      float ep = 0.f;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int c = wn * C::TN * 16 + j * 16 + cq;
        const float4 b = *reinterpret_cast<const float4*>(b2 + c);
        const float4 w = *reinterpret_cast<const float4*>(wo + c);
        float h[4], d[4];
        const float bb[4] = {b.x, b.y, b.z, b.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float z = acc[i][j][e] + bb[e];
          const float ex = __builtin_amdgcn_exp2f(fminf(z, 0.f) * ial2e);
          h[e] = rv ? (z > 0.f ? z : alpha * (ex - 1.f)) : 0.f;
          d[e] = rv ? up * ww[e] * (z > 0.f ? 1.f : ex) : 0.f;
          ep += ww[e] * h[e];
        }
        const float4 d4 = make_float4(d[0], d[1], d[2], d[3]);
        lds_put4(D3s + r * S3 + c * 2, d4);
        if (a.H3) Store<bf16_t>::put4(a.H3 + (size_t)row * W3 + c, make_float4(h[0], h[1], h[2], h[3]));
        if (a.D3) Store<bf16_t>::put4(a.D3 + (size_t)row * W3 + c, d4);
      }
      ep += __shfl_xor(ep, 16, 64);
      ep += __shfl_xor(ep, 32, 64);
      if (lane < 16) epart[wn * BM + r] = ep;
    }
  }
  __syncthreads();
  if (tid < BM) {
    const int row = row0 + tid;
    float e = a.bout[s];
#pragma unroll
    for (int q = 0; q < MidCfg<W3, BM>::WN; ++q) e += epart[q * BM + tid];
    if (row < row_end) a.erow[a.perm[row]] = e;  // input atom order
    if (a.uprow) {
      float up = 0.f;
      if (row < row_end) up = (a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f) * a.escale;
      a.uprow[row] = up;
    }
  }

  // ---- D2 = (D3 W2) * CELU'(z2), written over H2
  MidRing<W1, BM> br4;
  {
    using C = MidCfg<W2, BM>;
    f32x4_t acc[C::TM][C::TN];
    mid_steps<W2, W3, BM>(D3s, S3, br3, lane, wv, acc);
    mid_ring<W1, W2, BM>(br4, a.W1T + (size_t)s * W1 * W2, lane, wv);
    const int wm = wv / C::WN, wn = wv % C::WN;
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int r = wm * C::TM * 16 + i * 16 + rl;
      const bool rv = row0 + r < row_end;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int c = wn * C::TN * 16 + j * 16 + cq;
        const float4 h = lds_get4(X2 + r * S2 + c * 2);
        float4 d = make_float4(acc[i][j][0] * celu_slope(h.x, ia), acc[i][j][1] * celu_slope(h.y, ia),
                               acc[i][j][2] * celu_slope(h.z, ia), acc[i][j][3] * celu_slope(h.w, ia));
        if (!rv) d = make_float4(0.f, 0.f, 0.f, 0.f);
        lds_put4(X2 + r * S2 + c * 2, d);
        if (a.D2) Store<bf16_t>::put4(a.D2 + (size_t)(row0 + r) * W2 + c, d);
      }
    }
  }
  __syncthreads();

  // ---- D1 = (D2 W1) * CELU'(z1) -> global
  {
    using C = MidCfg<W1, BM>;
    const int wm = wv / C::WN, wn = wv % C::WN;
    const int ldd1 = a.ld_d1 ? a.ld_d1 : W1;
    // H1 for the slopes is fetched before the product (4 bf16 per tile)
    uint2 h1[C::TM][C::TN];
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int row = row0 + wm * C::TM * 16 + i * 16 + rl;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int c = wn * C::TN * 16 + j * 16 + cq;
        if (D3s != X1)  // H1 still in X1 (zero past the group)
          h1[i][j] = *reinterpret_cast<const uint2*>(X1 + (row - row0) * S1 + c * 2);
        else
          h1[i][j] = row < row_end
                         ? *reinterpret_cast<const uint2*>(a.H1 + (size_t)row * W1 + c)
                         : make_uint2(0, 0);
      }
    }
    f32x4_t acc[C::TM][C::TN];
    mid_steps<W1, W2, BM>(X2, S2, br4, lane, wv, acc);
    after_last();
#pragma unroll
    for (int i = 0; i < C::TM; ++i) {
      const int r = wm * C::TM * 16 + i * 16 + rl;
      const int row = row0 + r;
      const bool rv = row < row_end;
#pragma unroll
      for (int j = 0; j < C::TN; ++j) {
        const int c = wn * C::TN * 16 + j * 16 + cq;
        const uint2 u = h1[i][j];
        const float4 h = make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
        float4 d = make_float4(acc[i][j][0] * celu_slope(h.x, ia), acc[i][j][1] * celu_slope(h.y, ia),
                               acc[i][j][2] * celu_slope(h.z, ia), acc[i][j][3] * celu_slope(h.w, ia));
        if (!rv) d = make_float4(0.f, 0.f, 0.f, 0.f);
        if (d1_lds) lds_put4(d1_lds + r * S1 + c * 2, d);
        if (a.D1) Store<bf16_t>::put4(a.D1 + (size_t)row * ldd1 + c, d);
      }
    }
  }
}

template <int W1, int W2, int W3>
__global__ __launch_bounds__(512) void k_mlp_mid(MidArgs a) {
  static_assert(W3 <= W1, "D3 is stored over H1");
  constexpr int S1 = W1 * 2 + 16, S2 = W2 * 2 + 16;  // LDS row strides (bytes)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* X1 = smem;                          // H1, then D3
  unsigned char* X2 = X1 + kMidBM * S1;              // H2, then D2
  float* epart = reinterpret_cast<float*>(X2 + kMidBM * S2);  // [WN][128]

  const GroupTable* gt = a.gt;
  // tiles holding rows (groups are padded to whole tiles); the grid covers
  // the capacity, and blocks past the used tiles exit
  const int nt = gt->total_rows / kMidBM;
  if ((int)blockIdx.x >= nt) return;
  const int row0 = xcd_tile(blockIdx.x, nt) * kMidBM;
  const int s = tile_species(gt, row0);
  const int row_end = gt->pstart[s] + gt->cnt[s];
  if (row0 >= row_end) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // the first product's weights are requested before the H1 tile, so the
  // two latencies overlap
  MidRing<W2> br1;
  mid_ring<W2, W1>(br1, a.W1 + (size_t)s * W2 * W1, lane, wv);

  // H1 tile -> LDS (zero rows past the group): every load is issued before
  // the first store
  {
    constexpr int V1 = W1 / 8;  // 16-byte vectors per row
    constexpr int NV = kMidBM * V1 / 512;
    static_assert(kMidBM * V1 % 512 == 0, "whole vectors per thread");
    uint4 v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int idx = tid + q * 512, r = idx / V1, c = idx % V1;
      v[q] = make_uint4(0, 0, 0, 0);
      if (row0 + r < row_end)
        v[q] = *reinterpret_cast<const uint4*>(a.H1 + (size_t)(row0 + r) * W1 + c * 8);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int idx = tid + q * 512, r = idx / V1, c = idx % V1;
      *reinterpret_cast<uint4*>(X1 + r * S1 + c * 16) = v[q];
    }
  }
  __syncthreads();

  mid_products<W1, W2, W3, kMidBM>(a, br1, X1, X2, epart, row0, row_end, s, nullptr, X1, S1,
                                   [] {});
}

// ------------------------------------------------------------ whole network
//
// Layer 1, the fused middle and dE/dG for one tile of 64 species-sorted
// rows per workgroup of four waves, so H1 and D1 never make an HBM round
// trip and the three stages share one launch:
//   H1 = CELU(X W0^T + b0)      X streamed through two LDS chunk buffers
//                               (region A), weights through the register
//                               ring; H1 into LDS (X1), and to global
//                               memory only for the weight gradients
//   middle products             as k_mlp_mid, H2 / D2 and D3 in region A
//                               (H1 stays in X1 for the last slopes); D1
//                               into X1
//   G = D1 W0                   D1 resident in X1, passes of eight k-steps,
//                               staged per wave in region A for
//                               whole-row-segment stores
// Two workgroups share a CU (80 KB of LDS each, half of it), so one tile's
// barriers, epilogues and weight-ring latency overlap the other's products.
// Feature rows are sparse: an atom touches the blocks of the elements
// around it only (about an eighth of the row in the 64-atom conformations,
// the element pairs of water in a box).  With per-row masks of the k-steps
// (32 columns) that may be nonzero, a tile runs layer 1 and dE/dG over the
// union of its rows' k-steps only (a compacted k-step list, one entry per
// lane: about 60 % of the steps for the conformations), each row reads its
// own k-steps of X (the rest load as zero), and each row's dE/dG is written
// on its own k-steps only, which are all the symmetry-function adjoint
// reads.  The skipped steps would add exact zeros, so the results do not
// change.  LDS: region A (X2: 64 rows of 400 bytes, the energy partials
// (512 bytes) and D3: 64 rows of 336 bytes; during layer 1 the two chunk
// buffers, 34,816 bytes) + X1 (64 rows of 528 bytes) + the rows' masks (512
// bytes) = 81,920 bytes.
constexpr int kNetBM = 64;
constexpr int kNetThreads = 256;
constexpr int kNetChunk = 256;                  // bytes of K per row and chunk
constexpr int kNetChunkStride = kNetChunk + 16;

template <int W1, int W2, int W3>
struct NetLds {
  static constexpr int S1 = W1 * 2 + 16, S2 = W2 * 2 + 16, S3 = W3 * 2 + 16;
  static constexpr int EP = MidCfg<W3, kNetBM>::WN * kNetBM * 4;  // energy partials
  static constexpr int D3 = kNetBM * S2 + EP;                     // D3's offset
  static constexpr int RA_MID = D3 + kNetBM * S3;                 // region A in the middle
  static constexpr int RA_L1 = 2 * kNetBM * kNetChunkStride;      // ... during layer 1
  static constexpr int RA = RA_MID > RA_L1 ? RA_MID : RA_L1;
  static constexpr int X1 = RA;
  static constexpr int MASKS = X1 + kNetBM * S1;
  static constexpr size_t bytes = (size_t)MASKS + kNetBM * 8;
  static_assert(RA % 16 == 0 && D3 % 16 == 0, "aligned regions");
};

template <int W1, int W2, int W3>
constexpr size_t net_lds() {
  return NetLds<W1, W2, W3>::bytes;
}

template <int W1, int W2, int W3>
// (two workgroups per CU: at most 256 registers per lane)
__global__ __launch_bounds__(kNetThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mlp_net(
    MidArgs a) {
  using LL = NetLds<W1, W2, W3>;
  constexpr int BM = kNetBM, NTH = kNetThreads;
  constexpr int S1 = LL::S1;
  static_assert(LL::bytes * 2 <= 160 * 1024, "two workgroups per CU");
  static_assert(MidCfg<W1, BM>::WM * MidCfg<W1, BM>::WN * 64 == NTH, "the middle's waves");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  unsigned char* RAp = smem;
  unsigned char* X1 = smem + LL::X1;
  unsigned long long* rmask = reinterpret_cast<unsigned long long*>(smem + LL::MASKS);
  unsigned char* X2 = RAp;
  float* epart = reinterpret_cast<float*>(X2 + BM * LL::S2);
  unsigned char* D3s = smem + LL::D3;

  const GroupTable* gt = a.gt;
  const int nt = gt->total_rows / BM;
  if ((int)blockIdx.x >= nt) return;
  const int row0 = xcd_tile(blockIdx.x, nt) * BM;
  const int s = tile_species(gt, row0);
  const int row_end = gt->pstart[s] + gt->cnt[s];
  if (row0 >= row_end) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rl = lane & 15, cq = (lane >> 4) * 4;
  // layer 1 and dE/dG: each wave takes all 64 rows and a quarter of the
  // columns (A fragments from LDS, weight fragments once per workgroup)
  constexpr int WM = 1, WN = 4, TM = 4, TN = W1 / 64, P = 4;
  static_assert(WM * TM * 16 == BM && WN * TN * 16 == W1, "one pass covers layer 1");
  const int wm = wv / WN, wn = wv % WN;
  const int K = a.ldx;

  // ---- the tile's k-steps: the union of its rows' masks, compacted into
  // qlist (lane l: the l-th active k-step); rows past the group have none
  const int nks = K / Frag<bf16_t>::KS;
  const unsigned long long all = nks >= 64 ? ~0ull : (1ull << nks) - 1ull;
  auto row_mask = [&](int r) -> unsigned long long {
    if (!a.kmask) return all;
    return row0 + r < row_end ? a.kmask[row0 + r] & all : 0ull;
  };
  unsigned long long U;
  {
    static_assert(BM == 64, "one row per lane");
    const unsigned long long m = row_mask(lane);
    if (tid < BM) rmask[tid] = m;
    unsigned lo = (unsigned)m, hi = (unsigned)(m >> 32);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      lo |= __shfl_xor(lo, d, 64);
      hi |= __shfl_xor(hi, d, 64);
    }
    U = ((unsigned long long)__builtin_amdgcn_readfirstlane(hi) << 32) |
        (unsigned)__builtin_amdgcn_readfirstlane(lo);
  }
  const int nact = __popcll(U);
  const int qlist = nth_set_bit(U, lane);

  MidRing<W2, BM> br1;  // the middle's first product (started at layer 1's last step)
  // ---- layer 1: H1 = CELU(X W0^T + b0), over the active k-steps, four per
  // chunk; thread t loads 16-byte piece t % 4 of chunk slot (t / 4) % 4 of
  // rows t / 16 + 16 v
  {
    constexpr int KC = kNetChunk / 2;           // bf16 per chunk row
    constexpr int SPC = KC / Frag<bf16_t>::KS;  // k-steps per chunk
    static_assert(SPC == P, "one ring cycle per chunk");
    constexpr int VPR = kNetChunk / 16;
    constexpr int NVA = BM * VPR / NTH;
    constexpr int RPV = NTH / VPR;              // rows per round of loads
    static_assert(VPR == 16 && NVA == 4, "four rows per thread, a fixed piece of each");
    const __amdgpu_buffer_rsrc_t arsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<bf16_t*>(a.X + (size_t)row0 * K), (short)0, (row_end - row0) * K * 2,
        kBufferRsrcWord3);
    const int slot = (tid >> 2) & 3, piece = tid & 3;
    unsigned long long rm[NVA];
#pragma unroll
    for (int v = 0; v < NVA; ++v) rm[v] = row_mask((tid >> 4) + RPV * v);
    auto aload = [&](int c, uint4 (&ra)[NVA]) __attribute__((always_inline)) {
      const int pos = c * SPC + slot;
      const int q = __shfl(qlist, pos & 63, 64);
#pragma unroll
      for (int v = 0; v < NVA; ++v) {
        const int r = (tid >> 4) + RPV * v;
        const bool on = pos < nact && ((rm[v] >> q) & 1ull);
        const unsigned off = on ? (unsigned)((r * K + q * 32 + piece * 8) * 2) : kOutOfRange;
        const u32x4_t val = __builtin_amdgcn_raw_buffer_load_b128(arsrc, off, 0, 0);
        ra[v] = make_uint4(val[0], val[1], val[2], val[3]);
      }
    };
    auto astore = [&](int buf, const uint4 (&ra)[NVA]) __attribute__((always_inline)) {
      unsigned char* base = RAp + buf * BM * kNetChunkStride;
#pragma unroll
      for (int v = 0; v < NVA; ++v) {
        const int idx = tid + v * NTH;
        *reinterpret_cast<uint4*>(base + (idx / VPR) * kNetChunkStride + (idx % VPR) * 16) = ra[v];
      }
    };
    const int nu = nact > SPC ? (nact + SPC - 1) / SPC : 1;
    const int arow = (wm * TM * 16 + (lane & 15)) * kNetChunkStride + (lane >> 4) * 16;
    f32x4_t acc[TM][TN];
    zero_acc(acc);
    BRingQ<bf16_t, TN, P> br;
    br.init(a.W0 + (size_t)s * W1 * K, wn * TN * 16, lane, K, nact, qlist);
    br.prologue();
    uint4 ra0[NVA], ra1[NVA];
    aload(0, ra0);
    astore(0, ra0);
    aload(1 % nu, ra1);
    __syncthreads();
    auto unit = [&](int u, uint4 (&r_next2)[NVA], const uint4 (&r_next1)[NVA])
                    __attribute__((always_inline)) {
      aload(u + 2 < nu ? u + 2 : nu - 1, r_next2);
      kgroup<bf16_t, TM, TN, P>(RAp + (u & 1) * BM * kNetChunkStride + arow,
                                16 * kNetChunkStride, br, u * SPC, acc);
      astore((u + 1) & 1, r_next1);
      __syncthreads();
    };
    for (int u = 0; u < nu; u += 2) {
      unit(u, ra0, ra1);
      if (u + 1 < nu) unit(u + 1, ra1, ra0);
    }
    mid_ring<W2, W1, BM>(br1, a.W1 + (size_t)s * W2 * W1, lane, wv);
    const float alpha = a.alpha, ial2e = a.inv_alpha_l2e;
    const float* b0 = a.b0 + (size_t)s * W1;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int r = wm * TM * 16 + i * 16 + rl;
      const bool rv = row0 + r < row_end;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int c = wn * TN * 16 + j * 16 + cq;
        const float4 b = *reinterpret_cast<const float4*>(b0 + c);
        float4 h = make_float4(celu_fwd(acc[i][j][0] + b.x, alpha, ial2e),
                               celu_fwd(acc[i][j][1] + b.y, alpha, ial2e),
                               celu_fwd(acc[i][j][2] + b.z, alpha, ial2e),
                               celu_fwd(acc[i][j][3] + b.w, alpha, ial2e));
        if (!rv) h = make_float4(0.f, 0.f, 0.f, 0.f);
        lds_put4(X1 + r * S1 + c * 2, h);
        if (rv && a.D1) Store<bf16_t>::put4(a.H1out + (size_t)(row0 + r) * W1 + c, h);
      }
    }
  }
  __syncthreads();  // H1 in X1 (and in global memory); region A free

  // dE/dG (below): G = D1 W0 over the tile's active k-steps, eight per
  // pass: wave w takes positions 8 p + 2 w and 8 p + 2 w + 1 (column tiles
  // 2 q0, 2 q0 + 1, 2 q1, 2 q1 + 1) for all rows; its weight ring starts at
  // the middle's last product
  static_assert(TN == 4 && WN == 4, "two k-steps of 32 columns per wave and pass");
  const int npw = a.G && nact > 2 * wn ? (nact - 2 * wn + 7) / 8 : 0;  // this wave's passes
  auto qat = [&](int pos) -> int {
    return __builtin_amdgcn_readlane(qlist, pos < nact ? pos : (nact > 0 ? nact - 1 : 0));
  };
  const bf16_t* B = a.W0T + (size_t)s * K * W1;
  BRingPair<bf16_t, P> br;
  br.init(B, W1, lane, qat(2 * wn), qat(2 * wn + 1), qat(8 + 2 * wn), qat(8 + 2 * wn + 1));

  // ---- the middle: H2, energies, D3, D2, D1 (into X1)
  {
    MidArgs am = a;
    am.H1 = a.H1out;
    mid_products<W1, W2, W3, BM>(am, br1, X1, X2, epart, row0, row_end, s, X1, D3s, LL::S3, [&] {
      if (npw > 0) br.prologue();
    });
  }
  if (!a.G) return;  // block-uniform: no forces asked for
  __syncthreads();   // D1 in X1; region A free

  // ---- dE/dG
  {
    constexpr int SS = TN * 16 * 2 + 16;        // staging row stride (bytes)
    constexpr int VR = TN * 16 * 2 / 16;        // 16-byte vectors of a staged row
    static_assert(16 * VR % 64 == 0, "whole store rounds");
    const int arow = (wm * TM * 16 + (lane & 15)) * S1 + (lane >> 4) * 16;
    unsigned char* stg = RAp + wv * 16 * SS;
    f32x4_t acc[TM][TN];
    for (int p = 0; p < npw; ++p) {
      const int pos0 = 8 * p + 2 * wn;
      const bool two = pos0 + 1 < nact;
      const int q0 = qat(pos0), q1 = qat(pos0 + 1);
      zero_acc(acc);
#pragma unroll
      for (int c = 0; c < W1 / 128; ++c)
        kgroup<bf16_t, TM, TN, P>(X1 + arow + c * 256, 16 * S1, br, c * P, acc);
      br.next_pass(B, qat(pos0 + 16), qat(pos0 + 17), lane);
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int rloc = wm * TM * 16 + i * 16;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          lds_put4(stg + rl * SS + (j * 16 + cq) * 2,
                   make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]));
        wave_lds_sync();
#pragma unroll
        for (int u = 0; u < 16 * VR / 64; ++u) {
          const int idx = lane + u * 64;
          const int r = idx / VR, cv = idx % VR, h = cv >> 2;
          const int q = h ? q1 : q0;
          if ((h == 0 || two) && row0 + rloc + r < row_end && ((rmask[rloc + r] >> q) & 1ull)) {
            const uint4 val = *reinterpret_cast<const uint4*>(stg + r * SS + cv * 16);
            unsigned char* dst = reinterpret_cast<unsigned char*>(a.G) +
                                 ((size_t)(row0 + rloc + r) * K + q * 32 + (cv & 3) * 8) * 2;
            *reinterpret_cast<uint4*>(dst) = val;
          }
        }
        wave_lds_sync();
      }
    }
  }
}

template <int W1, int W2, int W3>
static size_t mid_lds() {
  return (size_t)kMidBM * ((W1 * 2 + 16) + (W2 * 2 + 16)) + 4 * kMidBM * sizeof(float);
}

template <int W1, int W2, int W3>
static void launch_mid_t(const MidArgs& a, int rows_cap, hipStream_t st) {
  const size_t lds = mid_lds<W1, W2, W3>();
  static const bool attr = (ensure_lds(k_mlp_mid<W1, W2, W3>), true);
  (void)attr;
  hipLaunchKernelGGL((k_mlp_mid<W1, W2, W3>), dim3(rows_cap / kMidBM), dim3(512), lds, st, a);
}

bool launch_mlp_net(const int* width, const MidArgs& a, int rows_cap, hipStream_t st) {
  if (!(width[1] == 256 && width[2] == 192 && width[3] == 160)) return false;
  if (a.ldx <= 0 || a.ldx % 256 != 0 || a.ldx > 2048 || !a.X || !a.W0 || !a.W0T || !a.H1out)
    return false;
  constexpr size_t lds = net_lds<256, 192, 160>();
  static const bool attr = (ensure_lds(k_mlp_net<256, 192, 160>), true);
  (void)attr;
  hipLaunchKernelGGL((k_mlp_net<256, 192, 160>), dim3(rows_cap / kNetBM), dim3(kNetThreads), lds,
                     st, a);
  return true;
}

// Widths with a fused kernel: 1008-256-192-160 (seven elements) and
// 384-160-128-96 (four elements).  Returns false for other widths.
bool launch_mlp_mid(const int* width, const MidArgs& a, int rows_cap, hipStream_t st) {
  if (width[1] == 256 && width[2] == 192 && width[3] == 160) {
    launch_mid_t<256, 192, 160>(a, rows_cap, st);
    return true;
  }
  if (width[1] == 160 && width[2] == 128 && width[3] == 96) {
    launch_mid_t<160, 128, 96>(a, rows_cap, st);
    return true;
  }
  return false;
}

}  // namespace nnp

// Per-element atomic networks as grouped GEMMs on MFMA.
//
// ANI potentials give each element its own network and sum the atomic
// outputs (Methods, "OpenMM-ML").  Atoms are sorted by element into groups
// that start at multiples of kPad rows, so one GEMM launch serves every
// element: a 128-row tile belongs to one group and uses that element's
// weights.  Layers are C = A * B^T with A the row-major activations and B a
// row-major [N][K] weight matrix (W for the forward pass, W^T copies for the
// adjoint).  Epilogues are fused:
//   CELU : h = CELU(acc + b)                                  (hidden layers)
//   HEAD : h3 = CELU(acc + b); E_i = w_out . h3 + b_out;
//          delta3 = upstream_i * w_out * CELU'(z3)             (last hidden layer)
//   BWD  : delta = acc * CELU'(z) with CELU'(z) = 1 + h/alpha for h <= 0
//   OUT  : plain output in the operand type (dE/dG)
// BF16 operands use v_mfma_f32_16x16x32_bf16 and FP32 operands
// v_mfma_f32_16x16x4f32; both accumulate in FP32.
#include "mfma_tile.h"

#include <type_traits>

namespace nnp {

// ------------------------------------------------------------- body layers
//
// One workgroup per 128-row tile (8 waves, WM x WN of TM x TN 16x16 tiles)
// covers all N columns in passes of NP = WN * TN * 16, so the activations
// are read from HBM once.  A moves through LDS in chunks of 256 bytes per
// row: up to three chunks (K <= 384 BF16 or 192 FP32) stay resident across
// the passes; longer K streams through two chunk buffers with two chunks in
// flight in registers.  Weights stream into registers P k-steps ahead, and
// across pass boundaries.  Each wave writes its results through a small LDS
// stage, 16 rows at a time, so that every store instruction writes whole
// 128-byte (BF16) or 256-byte (FP32) row segments.
constexpr int kChunkBytes = 256;
constexpr int kChunkStride = kChunkBytes + 16;  // LDS row stride (bytes)
constexpr int kMaxResident = 3;

template <typename T, int TN>
constexpr int stage_stride() { return TN * 16 * (int)sizeof(T) + 16; }

// KS (layer 1 with the feature rows' k-step masks, one pass over N): the
// K loop runs over the tile's compacted list of k-steps that some row has
// nonzero (the rows are whole, so the skipped steps are zero).
template <typename T, int WM, int WN, int TM, int TN, int EPI, bool RESIDENT, bool KS = false>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_rb(GemmArgs a) {
  constexpr int NT = 64 * WM * WN;
  constexpr int BM = WM * TM * 16;
  static_assert(BM == kPad, "a row tile is one padding unit of a species group");
  constexpr int NP = WN * TN * 16;
  constexpr int KC = kChunkBytes / sizeof(T);
  constexpr int SPC = KC / Frag<T>::KS;  // k-steps per chunk
  constexpr int P = 4;
  static_assert(SPC == P, "one ring cycle per chunk");
  constexpr int VPR = kChunkBytes / 16;
  constexpr int NVA = BM * VPR / NT;
  constexpr int SS = stage_stride<T, TN>();
  constexpr int WCOLB = TN * 16 * sizeof(T);  // bytes of a wave's tile row
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

  const GroupTable* gt = a.gt;
  // tiles holding rows (groups are padded to whole tiles); the grid covers
  // the capacity, and blocks past the used tiles exit
  const int nt = gt->total_rows / BM;
  if ((int)blockIdx.x >= nt) return;
  const int row0 = xcd_tile(blockIdx.x, nt) * BM;
  const int s = tile_species(gt, row0);
  const int row_end = gt->pstart[s] + gt->cnt[s];
  if (row0 >= row_end) return;  // a tile of pad rows only
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv % WN;
  const int K = a.K;
  const T* A = reinterpret_cast<const T*>(a.A);
  const T* B = reinterpret_cast<const T*>(a.Bq) + (size_t)s * a.sB;

  // KS: the union of the tile's rows' k-step masks, compacted into qlist
  // (lane l: the l-th active k-step)
  int nact = 0, qlist = 0;
  if constexpr (KS) {
    static_assert(sizeof(T) == 2 && BM <= NT, "BF16, one row per thread");
    __shared__ unsigned long long kun[NT / 64];
    const int nks = K / Frag<T>::KS;
    const unsigned long long all = nks >= 64 ? ~0ull : (1ull << nks) - 1ull;
    const unsigned long long m = tid < BM && row0 + tid < row_end ? a.kmask_k[row0 + tid] & all : 0ull;
    unsigned lo = (unsigned)m, hi = (unsigned)(m >> 32);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      lo |= __shfl_xor(lo, d, 64);
      hi |= __shfl_xor(hi, d, 64);
    }
    if (lane == 0) kun[wv] = ((unsigned long long)hi << 32) | lo;
    __syncthreads();
    unsigned long long U = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) U |= kun[w];
    nact = __popcll(U);
    qlist = nth_set_bit(U, lane);
  }

  // A is read through a buffer resource that spans exactly the tile's valid
  // rows: loads of pad rows, and of columns past K (sent past the range),
  // return zeros in hardware.  So no load sits behind a branch, which would
  // make the compiler assume it may not have been issued and let every later
  // wait for the weight ring also wait for one more ring slot.
  const __amdgpu_buffer_rsrc_t arsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<T*>(A + (size_t)row0 * a.lda), (short)0,
      (row_end - row0) * a.lda * (int)sizeof(T), kBufferRsrcWord3);
  auto aload = [&](int c, uint4 (&ra)[NVA]) __attribute__((always_inline)) {
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * NT;
      int r = idx / VPR, k = c * KC + (idx % VPR) * (16 / (int)sizeof(T));
      bool in = k < K;
      if constexpr (KS) {  // chunk slot (idx % VPR) / 4 holds position c * SPC + slot
        const int pos = c * SPC + (idx % VPR) / 4;
        k = __shfl(qlist, pos & 63, 64) * Frag<T>::KS + (idx % 4) * 8;
        in = pos < nact;
      }
      const unsigned off = in ? (unsigned)((r * a.lda + k) * (int)sizeof(T)) : kOutOfRange;
      const u32x4_t val = __builtin_amdgcn_raw_buffer_load_b128(arsrc, off, 0, 0);
      ra[v] = make_uint4(val[0], val[1], val[2], val[3]);
    }
  };
  auto astore = [&](int buf, const uint4 (&ra)[NVA]) __attribute__((always_inline)) {
    unsigned char* base = smem + buf * BM * kChunkStride;
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * NT;
      *reinterpret_cast<uint4*>(base + (idx / VPR) * kChunkStride + (idx % VPR) * 16) = ra[v];
    }
  };

  const int ns = KS ? nact : K / Frag<T>::KS;
  const int nchunks = ns > SPC ? (ns + SPC - 1) / SPC : 1;  // RESIDENT: <= kMaxResident
  const int npass = a.N / NP;
  const int arow = (wm * TM * 16 + (lane & 15)) * kChunkStride + (lane >> 4) * 16;
  const int rl = lane & 15, cq = (lane >> 4) * 4;
  const float* bias = a.bias ? a.bias + (size_t)s * a.sBias : nullptr;
  const float ia = 1.f / a.alpha;
  unsigned char* stg = smem + (RESIDENT ? nchunks : 2) * BM * kChunkStride + wv * 16 * SS;
  const int col_w = wn * TN * 16;  // this wave's first column inside a pass

  f32x4_t acc[TM][TN];
  zero_acc(acc);
  using Ring = std::conditional_t<KS, BRingQ<T, TN, P>, BRing<T, TN, P>>;
  Ring br;
  if constexpr (KS)
    br.init(B, col_w, lane, K, nact, qlist);
  else
    br.init(B, col_w, npass > 1 ? NP + col_w : -1, lane, K);
  br.prologue();

  // Epilogue of pass p: finish each 16x16 tile in registers (lane holds row
  // rl, columns cq..cq+3), stage 16 rows of the wave tile in LDS, then write
  // them as whole row segments.
  auto epilogue = [&](int p) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int rloc = wm * TM * 16 + i * 16;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = row0 + rloc + rl;
        const bool rv = row < row_end;
        const int col = p * NP + col_w + j * 16 + cq;
        float4 v = make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
        if constexpr (EPI == EPI_CELU) {
          const float4 b = *reinterpret_cast<const float4*>(bias + col);
          v = make_float4(celu_fwd(v.x + b.x, a.alpha, a.inv_alpha_l2e),
                          celu_fwd(v.y + b.y, a.alpha, a.inv_alpha_l2e),
                          celu_fwd(v.z + b.z, a.alpha, a.inv_alpha_l2e),
                          celu_fwd(v.w + b.w, a.alpha, a.inv_alpha_l2e));
        } else if constexpr (EPI == EPI_BWD) {
          if (rv) {
            const float4 h = Vec4<T>::get(reinterpret_cast<const T*>(a.H) + (size_t)row * a.ldh + col);
            v.x *= celu_slope(h.x, ia);
            v.y *= celu_slope(h.y, ia);
            v.z *= celu_slope(h.z, ia);
            v.w *= celu_slope(h.w, ia);
          }
        }
        if (!rv) v = make_float4(0.f, 0.f, 0.f, 0.f);
        Store<T>::put4(reinterpret_cast<T*>(stg + rl * SS + (j * 16 + cq) * sizeof(T)), v);
      }
      wave_lds_sync();
      // 16 rows x WCOLB bytes, 16 bytes per lane per store
      constexpr int VR = WCOLB / 16;  // vectors per row
#pragma unroll
      for (int q = 0; q < (16 * VR + 63) / 64; ++q) {
        const int idx = lane + q * 64;
        if (16 * VR % 64 == 0 || idx < 16 * VR) {
          const int r = idx / VR, cv = idx % VR;
          const uint4 val = *reinterpret_cast<const uint4*>(stg + r * SS + cv * 16);
          unsigned char* dst = reinterpret_cast<unsigned char*>(a.C) +
                               ((size_t)(row0 + rloc + r) * a.ldc + p * NP + col_w) * sizeof(T) +
                               cv * 16;
          *reinterpret_cast<uint4*>(dst) = val;
        }
      }
      wave_lds_sync();
    }
  };

  if constexpr (RESIDENT) {
    // every chunk's loads are in flight before the first LDS store
    uint4 ra[kMaxResident][NVA];
#pragma unroll
    for (int c = 0; c < kMaxResident; ++c)
      if (c < nchunks) aload(c, ra[c]);
#pragma unroll
    for (int c = 0; c < kMaxResident; ++c)
      if (c < nchunks) astore(c, ra[c]);
    __syncthreads();
    for (int p = 0; p < npass; ++p) {
      for (int c = 0; c < nchunks; ++c)
        kgroup<T, TM, TN, P>(smem + c * BM * kChunkStride + arow, 16 * kChunkStride, br, c * SPC,
                             acc);
      br.next_pass(B, p + 2 < npass ? (p + 2) * NP + col_w : -1, lane);
      epilogue(p);
      zero_acc(acc);
    }
  } else {
    // flat sequence of (pass, chunk) units u = p * nchunks + c; unit u + 1 is
    // in LDS-bound registers while unit u computes, unit u + 2 in flight
    const int nu = npass * nchunks;
    uint4 ra0[NVA], ra1[NVA];
    aload(0, ra0);
    astore(0, ra0);
    aload(1 % nchunks, ra1);
    __syncthreads();
    auto unit = [&](int u, uint4 (&r_next2)[NVA], const uint4 (&r_next1)[NVA])
                    __attribute__((always_inline)) {
      const int c = u % nchunks;
      aload((u + 2 < nu ? u + 2 : nu - 1) % nchunks, r_next2);
      kgroup<T, TM, TN, P>(smem + (u & 1) * BM * kChunkStride + arow, 16 * kChunkStride, br,
                           c * SPC, acc);
      astore((u + 1) & 1, r_next1);
      __syncthreads();
      if (c == nchunks - 1) {
        const int p = u / nchunks;
        br.next_pass(B, p + 2 < npass ? (p + 2) * NP + col_w : -1, lane);
        epilogue(p);
        zero_acc(acc);
      }
    };
    for (int u = 0; u < nu; u += 2) {
      unit(u, ra0, ra1);
      if (u + 1 < nu) unit(u + 1, ra1, ra0);
    }
  }
}

template <typename T, int WM, int WN, int TM, int TN, int EPI, bool RES>
static void launch_rb_t(const GemmArgs& a, int nchunks, int rows_cap, hipStream_t st) {
  const size_t lds = (size_t)(RES ? nchunks : 2) * kPad * kChunkStride +
                     (size_t)WM * WN * 16 * stage_stride<T, TN>();
  // layer 1 over the tile's nonzero k-steps: one pass over N, at most 64 steps
  if constexpr (EPI == EPI_CELU && sizeof(T) == 2) {
    if (a.kmask_k && a.N == WN * TN * 16 && a.K / Frag<T>::KS <= 64) {
      static const bool attr_ks = (ensure_lds(k_gemm_rb<T, WM, WN, TM, TN, EPI, RES, true>), true);
      (void)attr_ks;
      hipLaunchKernelGGL((k_gemm_rb<T, WM, WN, TM, TN, EPI, RES, true>), dim3(rows_cap / kPad),
                         dim3(64 * WM * WN), lds, st, a);
      return;
    }
  }
  static const bool attr = (ensure_lds(k_gemm_rb<T, WM, WN, TM, TN, EPI, RES>), true);
  (void)attr;
  hipLaunchKernelGGL((k_gemm_rb<T, WM, WN, TM, TN, EPI, RES>), dim3(rows_cap / kPad),
                     dim3(64 * WM * WN), lds, st, a);
}

template <typename T, int WM, int WN, int TM, int TN, int EPI>
static void launch_rb(const GemmArgs& a, int rows_cap, hipStream_t st) {
  const int nchunks = (int)((a.K * sizeof(T) + kChunkBytes - 1) / kChunkBytes);
  if (nchunks <= kMaxResident)
    launch_rb_t<T, WM, WN, TM, TN, EPI, true>(a, nchunks, rows_cap, st);
  else
    launch_rb_t<T, WM, WN, TM, TN, EPI, false>(a, nchunks, rows_cap, st);
}

// Column layout for N: 2 x 4 waves of 64-row x TN*16-column tiles when N is a
// multiple of 64 (passes of 64*TN, TN the largest of 4, 3, 2, 1 dividing
// N/64), else 4 x 2 waves of 32-row tiles with TN in 5, 3, 1.
template <typename T, int EPI>
static bool launch_body(const GemmArgs& a, int rows_cap, hipStream_t st) {
  if (a.K % Frag<T>::KS != 0) return false;
  if (a.N % 64 == 0) {
    if (a.N % 256 == 0) { launch_rb<T, 2, 4, 4, 4, EPI>(a, rows_cap, st); return true; }
    if (a.N % 192 == 0) { launch_rb<T, 2, 4, 4, 3, EPI>(a, rows_cap, st); return true; }
    if (a.N % 128 == 0) { launch_rb<T, 2, 4, 4, 2, EPI>(a, rows_cap, st); return true; }
    launch_rb<T, 2, 4, 4, 1, EPI>(a, rows_cap, st);
    return true;
  }
  if (a.N % 32 != 0) return false;
  if (a.N % 160 == 0) { launch_rb<T, 4, 2, 2, 5, EPI>(a, rows_cap, st); return true; }
  if (a.N % 96 == 0) { launch_rb<T, 4, 2, 2, 3, EPI>(a, rows_cap, st); return true; }
  launch_rb<T, 4, 2, 2, 1, EPI>(a, rows_cap, st);
  return true;
}

// ------------------------------------------------------- LDS-staged products
//
// The energy head (every column of a row in one workgroup: the energy is a
// dot product over them) and the FP32 layers, whose MFMA rate rather than
// latency bounds them: both operands are staged through a double-buffered
// LDS ring (128 bytes of K per row and stage, rows padded to 144 bytes), one
// barrier per stage, zero-filled K tail.  B is row-major [N][K] (ldb).
template <typename T> struct Mfma;
template <> struct Mfma<bf16_t> {
  static constexpr int BK = 64;    // K elements per LDS stage (128 bytes per row)
  static constexpr int RS = 72;    // LDS row stride in elements (144 bytes)
  static constexpr int KSUB = 2;   // fragment reads per stage
  // lane's element offset inside a stage for fragment read kk
  __device__ __forceinline__ static int koff(int lane, int kk) { return kk * 32 + (lane >> 4) * 8; }
  __device__ __forceinline__ static void mma(const uint4& a, const uint4& b, f32x4_t& acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                  __builtin_bit_cast(bf16x8_t, b), acc, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  static constexpr int BK = 32;
  static constexpr int RS = 36;
  static constexpr int KSUB = 2;
  // float4 read kk covers k = kk*16 + (lane>>4)*4 + {0..3}; component c feeds
  // MFMA c, whose four k slots (lane groups) are {c, 4+c, 8+c, 12+c} + kk*16
  __device__ __forceinline__ static int koff(int lane, int kk) { return kk * 16 + (lane >> 4) * 4; }
  __device__ __forceinline__ static void mma(const uint4& a, const uint4& b, f32x4_t& acc) {
    const float4 va = __builtin_bit_cast(float4, a);
    const float4 vb = __builtin_bit_cast(float4, b);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(va.x, vb.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(va.z, vb.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(va.w, vb.w, acc, 0, 0, 0);
  }
};

template <typename T, int BM, int BN>
constexpr size_t gemm_lds_bytes() {
  return (size_t)2 * (BM + BN) * Mfma<T>::RS * sizeof(T);
}

// 256 threads = WM x WN waves; wave tile (BM/WM) x (BN/WN) of 16x16 MFMA tiles.
template <typename T, int BM, int BN, int WM, int WN, int EPI>
__global__ __launch_bounds__(256) void k_gemm_lds(GemmArgs a) {
  static_assert(WM * WN == 4, "four waves");
  constexpr int BK = Mfma<T>::BK, RS = Mfma<T>::RS;
  constexpr int WTM = BM / WM, WTN = BN / WN;
  constexpr int TM = WTM / 16, TN = WTN / 16;
  static_assert(TM * 16 == WTM && TN * 16 == WTN, "wave tile must be whole 16x16 tiles");
  constexpr int VPR = BK * sizeof(T) / 16;     // 16-byte vectors per stage row (8)
  constexpr int EPV = 16 / sizeof(T);          // elements per vector
  constexpr int NVA = (BM * VPR + 255) / 256;  // vectors per thread, A
  constexpr int NVB = (BN * VPR + 255) / 256;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* As = reinterpret_cast<T*>(smem);
  T* Bs = As + 2 * BM * RS;

  const GroupTable* gt = a.gt;
  const int row0 = blockIdx.x * BM;
  if (row0 >= gt->total_rows) return;
  int s = 0;
#pragma unroll
  for (int q = 1; q < kMaxS; ++q) s = (row0 >= gt->pstart[q]) ? q : s;
  const int row_end = gt->pstart[s] + gt->cnt[s];
  if (row0 >= row_end) return;  // a tile of pad rows only
  const int n0 = blockIdx.y * BN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv % WN;

  const T* A = reinterpret_cast<const T*>(a.A);
  const T* B = reinterpret_cast<const T*>(a.B) + (size_t)s * a.sB;
  const int K = a.K;
  int nk = (K + BK - 1) / BK;

  // feature-row masks: the union over the tile's rows of their k-steps
  __shared__ unsigned long long kunion[4];
  __shared__ int klist[64];
  // (tiles whose stages or column blocks are not whole 32-column groups
  // ignore the masks and run every stage and block)
  constexpr bool kMaskable = BK == 32 && BN % 32 == 0;
  const unsigned long long* km = a.kmask_k ? a.kmask_k : a.kmask_n;
  const bool kskip = kMaskable && a.kmask_k && nk <= 64;
  unsigned jact = ~0u;  // dE/dG: this wave's 16-column tiles that some row reads
  if (kMaskable && km && (a.kmask_n || kskip)) {  // block-uniform
    static_assert(BM <= 256, "one row per thread");
    unsigned long long m = tid < BM && row0 + tid < row_end ? km[row0 + tid] : 0ull;
    unsigned lo = (unsigned)m, hi = (unsigned)(m >> 32);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      lo |= __shfl_xor(lo, d, 64);
      hi |= __shfl_xor(hi, d, 64);
    }
    if (lane == 0) kunion[wv] = ((unsigned long long)hi << 32) | lo;
    __syncthreads();
    const unsigned long long U = kunion[0] | kunion[1] | kunion[2] | kunion[3];
    if (a.kmask_n) {
      // this block's columns [n0, n0 + BN) in 32-column groups
      if (n0 / 32 + BN / 32 <= 64) {
        const unsigned long long gm = ((1ull << (BN / 32)) - 1ull) << (n0 / 32);
        if ((U & gm) == 0ull) return;  // no row of the tile reads these columns
        unsigned ja = 0;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if ((U >> ((n0 + wn * WTN + j * 16) >> 5)) & 1ull) ja |= 1u << j;
        jact = __builtin_amdgcn_readfirstlane(ja);
      }
    } else {
      const unsigned long long all = nk >= 64 ? ~0ull : (1ull << nk) - 1ull;
      const unsigned long long Uk = U & all;
      if (tid < 64 && ((Uk >> tid) & 1ull)) klist[__popcll(Uk & ((1ull << tid) - 1ull))] = tid;
      nk = __popcll(Uk);
      __syncthreads();
    }
  }
  // K stage kt covers columns [kcol(kt) * BK, + BK)
  auto kcol = [&](int kt) { return kskip ? klist[kt] : kt; };

  uint4 ra[NVA], rb[NVB];
  auto gload = [&](int kt) {
    const int k0 = kcol(kt) * BK;
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / VPR, sg = idx % VPR;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (idx < BM * VPR && row0 + r < row_end && k0 + sg * EPV < K)
        val = *reinterpret_cast<const uint4*>(A + (size_t)(row0 + r) * a.lda + k0 + sg * EPV);
      ra[v] = val;
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx / VPR, sg = idx % VPR;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (idx < BN * VPR && n0 + r < a.N && k0 + sg * EPV < K)
        val = *reinterpret_cast<const uint4*>(B + (size_t)(n0 + r) * a.ldb + k0 + sg * EPV);
      rb[v] = val;
    }
  };
  auto lstore = [&](int buf) {
    T* as = As + buf * BM * RS;
    T* bs = Bs + buf * BN * RS;
#pragma unroll
    for (int v = 0; v < NVA; ++v) {
      const int idx = tid + v * 256;
      if (idx < BM * VPR)
        *reinterpret_cast<uint4*>(as + (idx / VPR) * RS + (idx % VPR) * EPV) = ra[v];
    }
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      if (idx < BN * VPR)
        *reinterpret_cast<uint4*>(bs + (idx / VPR) * RS + (idx % VPR) * EPV) = rb[v];
    }
  };

  f32x4_t acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

  if (nk > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  const int rl = lane & 15;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    const T* as = As + buf * BM * RS + (wm * WTM + rl) * RS;
    const T* bs = Bs + buf * BN * RS + (wn * WTN + rl) * RS;
#pragma unroll
    for (int kk = 0; kk < Mfma<T>::KSUB; ++kk) {
      const int ko = Mfma<T>::koff(lane, kk);
      uint4 fa[TM], fb[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) fa[i] = *reinterpret_cast<const uint4*>(as + i * 16 * RS + ko);
#pragma unroll
      for (int j = 0; j < TN; ++j) fb[j] = *reinterpret_cast<const uint4*>(bs + j * 16 * RS + ko);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        // (dE/dG: columns no row of the tile reads are left at zero)
        if (EPI == EPI_OUT && !((jact >> j) & 1u)) continue;
#pragma unroll
        for (int i = 0; i < TM; ++i) Mfma<T>::mma(fa[i], fb[j], acc[i][j]);
      }
    }
    if (kt + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }

  // ------------------------------------------------------------- epilogue
  const float* bias = a.bias ? a.bias + (size_t)s * a.sBias : nullptr;
  const int rq = (lane >> 4) * 4;  // first of this lane's 4 rows inside a 16x16 tile
  if constexpr (EPI != EPI_HEAD) {
    // Stage the tile in LDS as float (CELU applied, or raw accumulators), then
    // write whole rows with one 4-column vector per thread and pass.
    constexpr int CS = BN + 4;
    static_assert((size_t)BM * CS * 4 <= gemm_lds_bytes<T, BM, BN>(), "staging fits");
    float* ct = reinterpret_cast<float*>(smem);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rloc = wm * WTM + i * 16 + rq + e;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int cloc = wn * WTN + j * 16 + rl;
          float v = acc[i][j][e];
          if constexpr (EPI == EPI_CELU) {
            const int col = n0 + cloc;
            v = celu_fwd(v + (col < a.N ? bias[col] : 0.f), a.alpha, a.inv_alpha_l2e);
          }
          ct[rloc * CS + cloc] = v;
        }
      }
    __syncthreads();
    constexpr int C4 = BN / 4;
    for (int idx = tid; idx < BM * C4; idx += 256) {
      const int rloc = idx / C4, c = (idx % C4) * 4;
      const int row = row0 + rloc, col = n0 + c;
      if (col >= a.N) continue;
      const bool rv = row < row_end;
      float4 v = *reinterpret_cast<const float4*>(ct + rloc * CS + c);
      if (!rv) v = make_float4(0.f, 0.f, 0.f, 0.f);
      if constexpr (EPI == EPI_BWD) {
        if (rv) {
          const T* hp = reinterpret_cast<const T*>(a.H) + (size_t)row * a.ldh + col;
          const float inv_a = 1.f / a.alpha;
          float h0 = Store<T>::get(hp), h1 = Store<T>::get(hp + 1), h2 = Store<T>::get(hp + 2),
                h3 = Store<T>::get(hp + 3);
          v.x *= h0 > 0.f ? 1.f : 1.f + h0 * inv_a;
          v.y *= h1 > 0.f ? 1.f : 1.f + h1 * inv_a;
          v.z *= h2 > 0.f ? 1.f : 1.f + h2 * inv_a;
          v.w *= h3 > 0.f ? 1.f : 1.f + h3 * inv_a;
        }
      }
      Store<T>::put4(reinterpret_cast<T*>(a.C) + (size_t)row * a.ldc + col, v);
    }
    return;
  } else {
    float epart[TM][4];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) epart[i][e] = 0.f;
    const float* wout = a.w_out + (size_t)s * a.sWout;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rloc = wm * WTM + i * 16 + rq + e;
        const int row = row0 + rloc;
        const bool rv = row < row_end;
        float up = 0.f;
        if (rv) up = (a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f) * a.escale;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int col = n0 + wn * WTN + j * 16 + rl;
          if (col >= a.N) continue;
          const float z = acc[i][j][e] + bias[col];
          const float ex = __builtin_amdgcn_exp2f(fminf(z, 0.f) * a.inv_alpha_l2e);
          const float h = z > 0.f ? z : a.alpha * (ex - 1.f);
          const float dh = z > 0.f ? 1.f : ex;
          if (rv) epart[i][e] += wout[col] * h;
          if (a.C)
            Store<T>::put(reinterpret_cast<T*>(a.C) + (size_t)row * a.ldc + col,
                          rv ? up * wout[col] * dh : 0.f);
          if (a.H3)
            Store<T>::put(reinterpret_cast<T*>(a.H3) + (size_t)row * a.ldh3 + col, rv ? h : 0.f);
        }
      }
    }
    // sum the 16 column lanes of each row, then the WN column slices (waves)
    float* part = reinterpret_cast<float*>(smem);  // [WN][BM], LDS reused after the K loop
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = group16_sum(epart[i][e]);
        if (rl == 0) part[wn * BM + wm * WTM + i * 16 + rq + e] = v;
      }
    __syncthreads();
    for (int t = tid; t < BM; t += 256) {
      const int row = row0 + t;
      float e = a.b_out[s];
#pragma unroll
      for (int q = 0; q < WN; ++q) e += part[q * BM + t];
      if (row < row_end) a.erow[a.perm[row]] = e;  // input atom order
      if (a.uprow) {
        float up = 0.f;
        if (row < row_end) up = (a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f) * a.escale;
        a.uprow[row] = up;
      }
    }
  }
}

// ------------------------------------------------------------ launch helpers

template <typename T, int BM, int BN, int WM, int WN, int EPI>
static void launch_tile(const GemmArgs& a, int rows_cap, hipStream_t st) {
  constexpr size_t lds = gemm_lds_bytes<T, BM, BN>();
  static const bool attr = (ensure_lds(k_gemm_lds<T, BM, BN, WM, WN, EPI>), true);
  (void)attr;
  dim3 grid((rows_cap + BM - 1) / BM, (a.N + BN - 1) / BN);
  hipLaunchKernelGGL((k_gemm_lds<T, BM, BN, WM, WN, EPI>), grid, dim3(256), lds, st, a);
}

// Column tile for the non-head layers: the largest of 128, 96, 80, 64, 32
// dividing N (all widths are multiples of 32).
static int gemm_pick_bn(int N, int epi) {
  if (epi == EPI_HEAD) return N;
  for (int bn : {128, 96, 80, 64, 32})
    if (N % bn == 0) return bn;
  return 0;
}

template <typename T, int EPI>
static bool launch_lds_body(const GemmArgs& a, int rows_cap, hipStream_t st) {
  switch (gemm_pick_bn(a.N, EPI)) {
    case 128: launch_tile<T, 128, 128, 2, 2, EPI>(a, rows_cap, st); return true;
    case 96: launch_tile<T, 128, 96, 2, 2, EPI>(a, rows_cap, st); return true;
    case 80: launch_tile<T, 128, 80, 4, 1, EPI>(a, rows_cap, st); return true;
    case 64: launch_tile<T, 128, 64, 2, 2, EPI>(a, rows_cap, st); return true;
    case 32: launch_tile<T, 128, 32, 2, 2, EPI>(a, rows_cap, st); return true;
    default: return false;
  }
}

// The head layer keeps every column of a row in one workgroup (the energy is
// a dot product over them): BN = N, 64-row tiles.
template <typename T>
static bool launch_head(const GemmArgs& a, int rows_cap, hipStream_t st) {
  switch (a.N) {
    case 96: launch_tile<T, 64, 96, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 128: launch_tile<T, 64, 128, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 160: launch_tile<T, 64, 160, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 192: launch_tile<T, 64, 192, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 224: launch_tile<T, 64, 224, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 256: launch_tile<T, 64, 256, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 32: launch_tile<T, 64, 32, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    case 64: launch_tile<T, 64, 64, 2, 2, EPI_HEAD>(a, rows_cap, st); return true;
    default: return false;
  }
}

// BF16 body layers use the register-streamed kernel (B in fragment order);
// FP32 body layers, whose MFMA rate rather than latency bounds them, and the
// head use the LDS-staged kernel (B row-major).
template <typename T>
bool launch_gemm(int epi, const GemmArgs& a, int rows_cap, hipStream_t st);
template <>
bool launch_gemm<bf16_t>(int epi, const GemmArgs& a, int rows_cap, hipStream_t st) {
  if (epi != EPI_HEAD && a.Bq == nullptr) return false;
  switch (epi) {
    case EPI_CELU: return launch_body<bf16_t, EPI_CELU>(a, rows_cap, st);
    case EPI_HEAD: return launch_head<bf16_t>(a, rows_cap, st);
    case EPI_BWD: return launch_body<bf16_t, EPI_BWD>(a, rows_cap, st);
    case EPI_OUT: return launch_body<bf16_t, EPI_OUT>(a, rows_cap, st);
  }
  return false;
}
template <>
bool launch_gemm<float>(int epi, const GemmArgs& a, int rows_cap, hipStream_t st) {
  switch (epi) {
    case EPI_CELU: return launch_lds_body<float, EPI_CELU>(a, rows_cap, st);
    case EPI_HEAD: return launch_head<float>(a, rows_cap, st);
    case EPI_BWD: return launch_lds_body<float, EPI_BWD>(a, rows_cap, st);
    case EPI_OUT: return launch_lds_body<float, EPI_OUT>(a, rows_cap, st);
  }
  return false;
}

// ------------------------------------------------------------ weight gradients
//
// dW[o][i] = sum over the element's rows of D[r][o] * H[r][i];  db[o] = sum D[r][o].
// The rows of each element are cut into chunks of `chunk` rows.  One launch
// writes every layer's partial sums per chunk, laid out like the element's
// flat parameter vector (layer by layer: W row-major, then b); a second adds
// the partials of each element in chunk order, so the result does not depend
// on scheduling.

constexpr int kWgVecMaxIn = 256;  // widest input of the vector output-layer path
struct WgLayerArgs {
  const void* D;
  const void* H;
  int ldd, ldh, Nout, Nin;
  int hgap0, hgap;  // input i >= hgap0 is column i + hgap of H
  int n_o, n_i;   // 128-wide output and input tiles
  int block0;     // first block of the layer after the output layer's
  long part_off;  // the layer's W inside a chunk's partial vector
};
struct WgVecArgs {
  const void* H;
  int ldh, Nin;
  long part_off;
};
struct WgNetArgs {
  const GroupTable* gt;
  int S, chunk;
  float* partial;
  long part_len;  // floats per chunk
  const float* up;
  WgVecArgs vec;
  int vec_blocks;    // a multiple of 8
  int tiled_blocks;  // MFMA tiles of all layers
  int n_tiled;
  WgLayerArgs L[kLayers];
};

// Any layer shape (VALU, 64 x 64 register outer products from 32-row LDS
// tiles): the fallback for widths the MFMA tiles do not take.
template <typename TD, typename TH>
__global__ __launch_bounds__(256) void k_wgrad(const GroupTable* __restrict__ gt, int S,
                                               const TD* __restrict__ D, int ldd, int Nout,
                                               const TH* __restrict__ H, int ldh, int Nin,
                                               int chunk, float* __restrict__ partial, long part_len,
                                               long part_off, int hgap0, int hgap) {
  __shared__ float sd[32][65];
  __shared__ float sh[32][65];
  const int c = blockIdx.x;
  if (c >= gt->n_wchunks) return;
  int s = 0;
  for (int q = 1; q < S; ++q) s = (c >= gt->wchunk[q]) ? q : s;
  const int r0 = gt->pstart[s] + (c - gt->wchunk[s]) * chunk;
  int r1 = r0 + chunk;
  const int rend = gt->pstart[s] + gt->cnt[s];
  r1 = r1 < rend ? r1 : rend;
  const int o0 = blockIdx.y * 64, i0 = blockIdx.z * 64;
  const int tid = threadIdx.x;
  const int to = (tid >> 4) * 4, ti = (tid & 15) * 4;
  float acc[4][4] = {};
  float bacc = 0.f;
  for (int r = r0; r < r1; r += 32) {
    for (int v = tid; v < 32 * 64; v += 256) {
      const int rr = v >> 6, cc = v & 63;
      const int row = r + rr;
      const bool ok = row < r1;
      sd[rr][cc] = (ok && o0 + cc < Nout) ? Store<TD>::get(D + (size_t)row * ldd + o0 + cc) : 0.f;
      const int hc = i0 + cc + (i0 + cc >= hgap0 ? hgap : 0);
      sh[rr][cc] = (ok && i0 + cc < Nin) ? Store<TH>::get(H + (size_t)row * ldh + hc) : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 32; ++rr) {
      float dv[4], hv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        dv[x] = sd[rr][to + x];
        hv[x] = sh[rr][ti + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += dv[x] * hv[y];
    }
    if (blockIdx.z == 0 && tid < 64) {
      for (int rr = 0; rr < 32; ++rr) bacc += sd[rr][tid];
    }
    __syncthreads();
  }
  float* out = partial + (size_t)c * part_len + part_off;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int o = o0 + to + x, i = i0 + ti + y;
      if (o < Nout && i < Nin) out[(size_t)o * Nin + i] = acc[x][y];
    }
  if (blockIdx.z == 0 && tid < 64 && o0 + tid < Nout) out[(size_t)Nout * Nin + o0 + tid] = bacc;
}

constexpr int kWgBO = 128, kWgBI = 128;

template <typename T> struct WgLayout;
template <> struct WgLayout<bf16_t> {
  static constexpr int BK = 64;                 // atom rows per stage
  static constexpr int P = 72;                  // elements per LDS row (144 bytes)
  static constexpr int TILE = 128 * P;          // elements per operand tile
  // element (c, k): row c of the transposed tile (an output or input), atom
  // row k of the stage; 8-row granules XOR-swizzled by (c / 16) % 8
  __device__ __forceinline__ static int off(int c, int k) {
    return c * P + 8 * ((k >> 3) ^ ((c >> 4) & 7)) + (k & 7);
  }
};
template <> struct WgLayout<float> {
  static constexpr int BK = 32;
  static constexpr int RS = 144;                // floats per LDS row (one atom row)
  static constexpr int TILE = BK * RS;
  static constexpr int ITEMS = BK * 32 / 256;
};

template <typename T>
constexpr size_t wgrad_lds_bytes() {
  return (size_t)2 * 2 * WgLayout<T>::TILE * sizeof(T);
}


// The MFMA partials of one (chunk, 128 o, 128 i) tile, as C[i][o] = sum_r
// H[r][i] D[r][o] with K = the chunk's rows; four waves of 64 x 64 (4 x 4
// MFMA tiles).  Every stage reads BK rows of D and H with coalesced 16-byte
// loads into registers two stages ahead of the one being multiplied, so two
// stages' loads are in flight behind each stage's products.  The loads go
// through buffer resources that start at the stage's first row and end at
// the chunk's last: rows past the chunk, and columns past the layer (sent out
// of range), load as zeros, and no load sits behind a branch.
//   FP32 (v_mfma_f32_16x16x4f32, one K element per lane): the rows stay
//   row-major in LDS (144 floats per row, so the four K rows of a fragment
//   fall in different banks), and a fragment is one 4-byte read per lane.
//   BF16 (v_mfma_f32_16x16x32_bf16, eight consecutive K per lane): waves 0-1
//   stage D and waves 2-3 H; each thread loads an 8-row x 8-column block
//   (eight 16-byte row pieces), transposes it in registers (byte permutes)
//   and stores eight 16-byte column pieces, each one MFMA K granule, into a
//   transposed tile: one LDS row per output (or input) holding the stage's
//   64 atom rows, rows 144 bytes apart, granules XOR-swizzled by (c / 16) % 8.
//   Then neither the stores nor the fragment reads meet two to a bank
//   (16 lanes per pass of a 16-byte access, 64 banks; a CPU model of the
//   layout checks every instruction).
// Tiles at i = 0 also sum db: each thread adds the D columns it loads over
// its rows in registers, and the threads of a column group are added in a
// fixed order at the end.  The accumulator layout leaves each lane four
// consecutive i of one o, stored as one vector.
template <typename T>
__device__ __forceinline__ void wgrad_tile(const T* __restrict__ D, int ldd, int Nout,
                                           const T* __restrict__ H, int ldh, int Nin, int hgap0,
                                           int hgap, int r0, int r1, int o0, int i0, bool bias,
                                           float* __restrict__ out, float* __restrict__ bout,
                                           T* lds) {
  using L = WgLayout<T>;
  constexpr bool BF = sizeof(T) == 2;
  constexpr int BK = L::BK;
  constexpr int NL = 8;  // 16-byte loads per thread and stage
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wo = w >> 1, wi = w & 1;  // this wave's 64 x 64 tile

  // BF16: this thread's block (operand op, column group g, row block blk);
  // FP32: item k is atom row (tid + 256 k) / 32 (both operands), columns
  // 4 (tid % 32) .. + 3.
  const int op = __builtin_amdgcn_readfirstlane(w >> 1);  // BF16: 0 stages D, 1 H
  const int bu = tid & 127, bg = bu & 15, blk = bu >> 4;
  unsigned offs[NL];
  constexpr int NB = BF ? 8 : 4;  // columns per thread summed for db
  float bsum[NB];
#pragma unroll
  for (int e = 0; e < NB; ++e) bsum[e] = 0.f;
  if constexpr (BF) {
    const int ld = op ? ldh : ldd, N = op ? Nin : Nout, c = (op ? i0 : o0) + 8 * bg;
    const int cm = c + (op && c >= hgap0 ? hgap : 0);  // (8-column groups: the gap is too)
#pragma unroll
    for (int e = 0; e < NL; ++e)
      offs[e] = c < N ? (unsigned)(((8 * blk + e) * ld + cm) * 2) : kOutOfRange;
  } else {
    const int g = tid & 31, oc = o0 + 4 * g, ic = i0 + 4 * g;
#pragma unroll
    for (int k = 0; k < NL / 2; ++k) {
      const int r = (tid >> 5) + 8 * k;
      offs[k] = oc < Nout ? (unsigned)((r * ldd + oc) * 4) : kOutOfRange;
      offs[NL / 2 + k] =
          ic < Nin ? (unsigned)((r * ldh + ic + (ic >= hgap0 ? hgap : 0)) * 4) : kOutOfRange;
    }
  }
  uint4 ra0[NL], ra1[NL];
  auto gload = [&](uint4 (&ra)[NL], int rb) __attribute__((always_inline)) {
    // (uniform; read into a scalar register so that the resources are built
    // there and the loads need no per-lane resource loop)
    const int nr = __builtin_amdgcn_readfirstlane(r1 - rb < 0 ? 0 : (r1 - rb < BK ? r1 - rb : BK));
    const __amdgpu_buffer_rsrc_t dsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(D + (size_t)rb * ldd), (short)0, nr * ldd * (int)sizeof(T),
        kBufferRsrcWord3);
    const __amdgpu_buffer_rsrc_t hsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(H + (size_t)rb * ldh), (short)0, nr * ldh * (int)sizeof(T),
        kBufferRsrcWord3);
#pragma unroll
    for (int e = 0; e < NL; ++e) {
      u32x4_t v;
      if constexpr (BF)
        v = __builtin_amdgcn_raw_buffer_load_b128(op ? hsrc : dsrc, offs[e], 0, 0);
      else
        v = __builtin_amdgcn_raw_buffer_load_b128(e < NL / 2 ? dsrc : hsrc, offs[e], 0, 0);
      ra[e] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  };
  auto addbias = [&](const uint4 (&ra)[NL]) __attribute__((always_inline)) {
    if constexpr (BF) {
      if (op != 0) return;
#pragma unroll
      for (int e = 0; e < NL; ++e) {
        const unsigned u[4] = {ra[e].x, ra[e].y, ra[e].z, ra[e].w};
#pragma unroll
        for (int c = 0; c < 8; ++c)
          bsum[c] += __uint_as_float((c & 1) ? (u[c >> 1] & 0xffff0000u) : (u[c >> 1] << 16));
      }
    } else {
#pragma unroll
      for (int k = 0; k < NL / 2; ++k) {
        bsum[0] += __uint_as_float(ra[k].x);
        bsum[1] += __uint_as_float(ra[k].y);
        bsum[2] += __uint_as_float(ra[k].z);
        bsum[3] += __uint_as_float(ra[k].w);
      }
    }
  };
  auto lstore = [&](const uint4 (&ra)[NL], int buf) __attribute__((always_inline)) {
    T* dt = lds + (size_t)buf * 2 * L::TILE;
    if constexpr (BF) {
      // column c of the block: (row 2q, row 2q + 1) pairs from the low
      // (c even) or high (c odd) halves of dword c / 2 of rows 2q and 2q + 1
      T* tile = dt + op * L::TILE;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const unsigned sel = (c & 1) ? 0x07060302u : 0x05040100u;
        unsigned q[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const uint4 a = ra[2 * h], b = ra[2 * h + 1];
          const unsigned ua[4] = {a.x, a.y, a.z, a.w}, ub[4] = {b.x, b.y, b.z, b.w};
          q[h] = __builtin_amdgcn_perm(ub[c >> 1], ua[c >> 1], sel);
        }
        *reinterpret_cast<uint4*>(tile + L::off(8 * bg + c, 8 * blk)) =
            make_uint4(q[0], q[1], q[2], q[3]);
      }
    } else {
      T* ht = dt + L::TILE;
#pragma unroll
      for (int k = 0; k < NL / 2; ++k) {
        const int r = (tid >> 5) + 8 * k, g = tid & 31;
        *reinterpret_cast<uint4*>(dt + r * L::RS + g * 4) = ra[k];
        *reinterpret_cast<uint4*>(ht + r * L::RS + g * 4) = ra[NL / 2 + k];
      }
    }
  };
  f32x4_t acc[4][4];
  zero_acc(acc);
  auto compute = [&](int buf) __attribute__((always_inline)) {
    const T* dt = lds + (size_t)buf * 2 * L::TILE;
    const T* ht = dt + L::TILE;
    if constexpr (BF) {
#pragma unroll 1
      for (int kk = 0; kk < 2; ++kk) {
        const int j = kk * 4 + (lane >> 4);  // this lane's 8-row granule
        uint4 fa[4], fb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int ci = wi * 64 + x * 16 + (lane & 15);
          fa[x] = *reinterpret_cast<const uint4*>(ht + L::off(ci, 8 * j));
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int co = wo * 64 + y * 16 + (lane & 15);
          fb[y] = *reinterpret_cast<const uint4*>(dt + L::off(co, 8 * j));
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) Mfma<bf16_t>::mma(fa[x], fb[y], acc[x][y]);
      }
    } else {
#pragma unroll 2
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        float fa[4], fb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) fa[x] = ht[kr * L::RS + wi * 64 + x * 16 + (lane & 15)];
#pragma unroll
        for (int y = 0; y < 4; ++y) fb[y] = dt[kr * L::RS + wo * 64 + y * 16 + (lane & 15)];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[x], fb[y], acc[x][y], 0, 0, 0);
      }
    }
  };

  // Stage s is loaded into register set s % 2 two stages before it is
  // multiplied and stored to LDS buffer s % 2 one stage before.  The stage
  // count is rounded up to even and every load is issued: stages past the
  // chunk read an empty range (zeros, which add nothing), so no load sits
  // behind a branch and each wait covers exactly the set it needs.
  const int nst = (r1 - r0 + 2 * BK - 1) / (2 * BK) * 2;
  gload(ra0, r0);
  gload(ra1, r0 + BK);
  if (bias) addbias(ra0);
  lstore(ra0, 0);
  gload(ra0, r0 + 2 * BK);
  __syncthreads();
  for (int st = 0; st < nst; st += 2) {
    compute(0);
    if (bias) addbias(ra1);
    lstore(ra1, 1);
    gload(ra1, r0 + (st + 3) * BK);
    __syncthreads();
    compute(1);
    if (bias) addbias(ra0);
    lstore(ra0, 0);
    gload(ra0, r0 + (st + 4) * BK);
    __syncthreads();
  }
  // acc[x][y][e]: i = i0 + wi 64 + x 16 + 4 (lane / 16) + e, o = o0 + wo 64 + y 16 + lane % 16
  const int iq = 4 * (lane >> 4);
#pragma unroll
  for (int y = 0; y < 4; ++y) {
    const int o = o0 + wo * 64 + y * 16 + (lane & 15);
    if (o >= Nout) continue;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int i = i0 + wi * 64 + x * 16 + iq;
      if (i < Nin)
        *reinterpret_cast<float4*>(out + (size_t)o * Nin + i) =
            make_float4(acc[x][y][0], acc[x][y][1], acc[x][y][2], acc[x][y][3]);
    }
  }
  if (bias) {
    // the LDS tiles are free after the loop's last barrier; red[q][o] holds
    // the column sums of the q-th group of threads covering output o
    float* red = reinterpret_cast<float*>(lds);
    constexpr int NG = BF ? 8 : 8;
    if constexpr (BF) {
      if (op == 0) {
#pragma unroll
        for (int c = 0; c < 8; ++c) red[blk * 128 + 8 * bg + c] = bsum[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) red[(tid >> 5) * 128 + 4 * (tid & 31) + c] = bsum[c];
    }
    __syncthreads();
    if (tid < 128 && o0 + tid < Nout) {
      float v = 0.f;
      for (int q = 0; q < NG; ++q) v += red[q * 128 + tid];
      bout[o0 + tid] = v;
    }
  }
}

// The output layer's partials (one output): dW[i] = sum_r up[r] H[r][i],
// db = sum_r up[r].  Lane l takes columns 4l..4l+3 of every row (one 8- or
// 16-byte load), the workgroup's four waves take 16-row blocks in turn, and
// the 16 rows' loads are issued together through buffer resources spanning
// the chunk (rows past it and columns past Nin load as zeros, so no load is
// behind a branch).  The waves' sums are added in wave order.
template <typename TH>
__device__ __forceinline__ void wgrad_vec(const float* __restrict__ up,
                                          const TH* __restrict__ H, int ldh, int Nin, int r0,
                                          int r1, float* __restrict__ out, float* red) {
  constexpr int U = 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nrow = __builtin_amdgcn_readfirstlane(r1 - r0);
  const __amdgpu_buffer_rsrc_t hs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<TH*>(H + (size_t)r0 * ldh), (short)0, nrow * ldh * (int)sizeof(TH),
      kBufferRsrcWord3);
  const __amdgpu_buffer_rsrc_t us = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(up + r0), (short)0, nrow * 4, kBufferRsrcWord3);
  const int c0 = 4 * lane;
  const bool cok = c0 < Nin;
  float acc[4] = {0.f, 0.f, 0.f, 0.f}, bacc = 0.f;
  for (int rb = w * U; rb < nrow; rb += 4 * U) {
    float d[U], hv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + u;
      d[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(us, r * 4, 0, 0));
      const unsigned off = cok ? (unsigned)((r * ldh + c0) * (int)sizeof(TH)) : kOutOfRange;
      if constexpr (sizeof(TH) == 2) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(hs, off, 0, 0);
        hv[u][0] = __uint_as_float(v[0] << 16);
        hv[u][1] = __uint_as_float(v[0] & 0xffff0000u);
        hv[u][2] = __uint_as_float(v[1] << 16);
        hv[u][3] = __uint_as_float(v[1] & 0xffff0000u);
      } else {
        const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(hs, off, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) hv[u][e] = __uint_as_float(v[e]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      bacc += d[u];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += d[u] * hv[u][e];
    }
  }
  constexpr int RS = kWgVecMaxIn + 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) red[w * RS + c0 + e] = acc[e];
  if (lane == 0) red[w * RS + kWgVecMaxIn] = bacc;
  __syncthreads();
  for (int i = threadIdx.x; i <= Nin; i += 256) {
    const int src = i < Nin ? i : kWgVecMaxIn;
    out[i] = ((red[src] + red[RS + src]) + red[2 * RS + src]) + red[3 * RS + src];
  }
}

// Which (element, row range) chunk c covers; false past the last chunk.
__device__ __forceinline__ bool wgrad_chunk(const GroupTable* gt, int S, int chunk, int c,
                                            int& r0, int& r1) {
  if (c >= gt->n_wchunks) return false;
  int s = 0;
  for (int q = 1; q < S; ++q) s = (c >= gt->wchunk[q]) ? q : s;
  r0 = gt->pstart[s] + (c - gt->wchunk[s]) * chunk;
  const int rend = gt->pstart[s] + gt->cnt[s];
  r1 = r0 + chunk < rend ? r0 + chunk : rend;
  return true;
}

// Blocks [0, vec_blocks) take the output layer's chunks; then, layer by
// layer, (chunk, o-tile, i-tile) MFMA tiles, chunk-major.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_wgrad_net(
    WgNetArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  int b = blockIdx.x;
  int r0 = 0, r1 = 0;
  if (b < a.vec_blocks) {
    if (!wgrad_chunk(a.gt, a.S, a.chunk, b, r0, r1)) return;
    wgrad_vec<T>(a.up, static_cast<const T*>(a.vec.H), a.vec.ldh, a.vec.Nin, r0, r1,
                 a.partial + (size_t)b * a.part_len + a.vec.part_off,
                 reinterpret_cast<float*>(smem));
    return;
  }
  // Tiles in XCD-major order: workgroups are dealt to the eight XCDs in
  // turn, so physical block b (after the 8-aligned output-layer blocks) is
  // slot b / 8 on XCD b % 8; XCD x takes the contiguous range of tiles
  // [x, x + 1) * T / 8, which keeps the tiles of one chunk (reading the same
  // rows of D and H) on one XCD and its L2.
  b -= a.vec_blocks;
  {
    const int per_xcd = (a.tiled_blocks + 7) / 8;
    b = (b % 8) * per_xcd + b / 8;
    if (b >= a.tiled_blocks) return;
  }
  int l = 0;
  for (int q = 1; q < a.n_tiled; ++q) l = b >= a.L[q].block0 ? q : l;
  const WgLayerArgs& Ly = a.L[l];
  b -= Ly.block0;
  const int per = Ly.n_o * Ly.n_i;
  const int c = b / per, t = b % per;
  const int ot = t / Ly.n_i, it = t % Ly.n_i;
  if (!wgrad_chunk(a.gt, a.S, a.chunk, c, r0, r1)) return;
  float* out = a.partial + (size_t)c * a.part_len + Ly.part_off;
  wgrad_tile<T>(static_cast<const T*>(Ly.D), Ly.ldd, Ly.Nout, static_cast<const T*>(Ly.H), Ly.ldh,
                Ly.Nin, Ly.hgap0, Ly.hgap, r0, r1, ot * kWgBO, it * kWgBI, it == 0, out,
                out + (size_t)Ly.Nout * Ly.Nin, reinterpret_cast<T*>(smem));
}

// out[s] (W then b, Nout*Nin + Nout floats at param_off[s]) = sum of partials.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const GroupTable* __restrict__ gt, int S,
                                                      const float* __restrict__ partial, long len,
                                                      float* __restrict__ dparams,
                                                      const long* __restrict__ param_off) {
  const int s = blockIdx.y;
  if (s >= S) return;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  float v = 0.f;
  for (int c = gt->wchunk[s]; c < gt->wchunk[s + 1]; ++c) v += partial[(size_t)c * len + e];
  dparams[param_off[s] + e] = v;
}

template <typename T>
void launch_wgrad_net(const GroupTable* gt, int S, int n_chunks_cap, int chunk,
                      const WgradLayer* layers, int n_layers, float* partial, float* dparams,
                      const long* param_off_dev, hipStream_t st) {
  if (n_chunks_cap <= 0 || n_layers <= 0) return;
  static const bool attr = (ensure_lds(k_wgrad_net<T>), true);
  (void)attr;
  long part_len = 0, off[kLayers] = {};
  for (int l = 0; l < n_layers; ++l) {
    off[l] = part_len;
    part_len += (long)layers[l].Nout * layers[l].Nin + layers[l].Nout;
  }
  WgNetArgs a{};
  a.gt = gt;
  a.S = S;
  a.chunk = chunk;
  a.partial = partial;
  a.part_len = part_len;
  int blocks = 0;
  // the output layer: the vector kernel when it has one output
  const WgradLayer& lo = layers[n_layers - 1];
  const bool vec = lo.Nout == 1 && lo.Nin <= kWgVecMaxIn && lo.Nin % 4 == 0 && lo.ldh % 4 == 0;
  if (vec) {
    a.up = static_cast<const float*>(lo.D);
    a.vec.H = lo.H;
    a.vec.ldh = lo.ldh;
    a.vec.Nin = lo.Nin;
    a.vec.part_off = off[n_layers - 1];
    a.vec_blocks = (n_chunks_cap + 7) / 8 * 8;
  }
  for (int l = 0; l < n_layers; ++l) {
    const WgradLayer& y = layers[l];
    if (l == n_layers - 1 && vec) continue;
    const bool tiled = y.Nout >= 16 && y.Nout % 4 == 0 && y.Nin % 4 == 0 && y.ldd % 8 == 0 &&
                       y.ldh % 8 == 0 && !y.d_fp32;
    if (tiled && a.n_tiled < kLayers) {
      WgLayerArgs& t = a.L[a.n_tiled++];
      t.D = y.D; t.H = y.H; t.ldd = y.ldd; t.ldh = y.ldh; t.Nout = y.Nout; t.Nin = y.Nin;
      t.hgap0 = y.hgap0; t.hgap = y.hgap;
      t.n_o = (y.Nout + kWgBO - 1) / kWgBO;
      t.n_i = (y.Nin + kWgBI - 1) / kWgBI;
      t.block0 = blocks;
      t.part_off = off[l];
      blocks += n_chunks_cap * t.n_o * t.n_i;
    } else if (y.d_fp32) {
      dim3 grid(n_chunks_cap, (y.Nout + 63) / 64, (y.Nin + 63) / 64);
      hipLaunchKernelGGL((k_wgrad<float, T>), grid, dim3(256), 0, st, gt, S,
                         static_cast<const float*>(y.D), y.ldd, y.Nout,
                         static_cast<const T*>(y.H), y.ldh, y.Nin, chunk, partial, part_len,
                         off[l], y.hgap0, y.hgap);
    } else {
      dim3 grid(n_chunks_cap, (y.Nout + 63) / 64, (y.Nin + 63) / 64);
      hipLaunchKernelGGL((k_wgrad<T, T>), grid, dim3(256), 0, st, gt, S,
                         static_cast<const T*>(y.D), y.ldd, y.Nout, static_cast<const T*>(y.H),
                         y.ldh, y.Nin, chunk, partial, part_len, off[l], y.hgap0, y.hgap);
    }
  }
  a.tiled_blocks = blocks;
  const int total = a.vec_blocks + (blocks + 7) / 8 * 8;
  if (total > 0)
    hipLaunchKernelGGL(k_wgrad_net<T>, dim3(total), dim3(256), wgrad_lds_bytes<T>(), st, a);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((part_len + 255) / 256), S), dim3(256), 0,
                     st, gt, S, partial, part_len, dparams, param_off_dev);
}
template void launch_wgrad_net<float>(const GroupTable*, int, int, int, const WgradLayer*, int,
                                      float*, float*, const long*, hipStream_t);
template void launch_wgrad_net<bf16_t>(const GroupTable*, int, int, int, const WgradLayer*, int,
                                       float*, float*, const long*, hipStream_t);

// ------------------------------------------------------------ weight packing
//
// From the flat parameter vector (per species, per layer: W row-major
// out x in, then b) to: W_l [S][out][in_pad] row-major (float and bf16) and
// W_l^T [S][in_pad][out] row-major (float), the LDS-staged kernels' operands;
// W_l and W_l^T in MFMA fragment order (bf16), the register-streamed
// kernels' operands; biases [S][out], output weights [S][w3] and output
// biases [S].  One thread per (species, layer, out, in_pad).
//
// Fragment order of a [N][K] operand: 16-row tiles, then k-steps of KS, then
// the 64 lanes of the wave, then the EL elements of a lane; lane l of k-step
// ks in tile nt holds row nt*16 + l % 16, columns ks*KS + (l / 16)*EL + e.
// A wave's fragment is then one contiguous 1 KB block.
template <typename T>
__device__ __forceinline__ size_t frag_off(int n, int k, int K) {
  constexpr int KS = Frag<T>::KS, EL = Frag<T>::EL;
  const int kk = k % KS;
  const int lane = (kk / EL) * 16 + n % 16;
  return (((size_t)(n / 16) * (K / KS) + k / KS) * 64 + lane) * EL + kk % EL;
}

__global__ __launch_bounds__(256) void k_pack(PackArgs p) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y, s = blockIdx.z;  // s: weight slot (member * S + element)
  const int in = p.width[l], out = p.width[l + 1];
  const int inp = l == 0 ? p.Fp : in;
  const float* src = p.flat + p.off[s * kLayers + l];
  if (l < kLayers - 1) {
    if (t >= (long)out * inp) return;
    const int o = (int)(t / inp), i = (int)(t % inp);
    // layer 1: inputs from r0 on sit at columns from a0 on (zero between)
    const int pi = l == 0 && i >= p.r0 ? i - (p.a0 - p.r0) : i;
    const bool on = pi < in && (l != 0 || i < p.r0 || i >= p.a0);
    const float v = on ? src[(size_t)o * in + pi] : 0.f;
    const size_t ws = (size_t)s * out * inp;
    p.Wf[l][ws + (size_t)o * inp + i] = v;
    p.Wb[l][ws + (size_t)o * inp + i] = f2bf(v);
    p.WTf[l][ws + (size_t)i * out + o] = v;
    p.Wqb[l][ws + frag_off<bf16_t>(o, i, inp)] = f2bf(v);
    p.WTqb[l][ws + frag_off<bf16_t>(i, o, out)] = f2bf(v);
    if (i == 0) p.bias[l][(size_t)s * out + o] = src[(size_t)out * in + o];
    if (l == 0 && p.n_models > 1) {
      // member k's W_0^T as columns [k out, (k + 1) out) of one K = M out operand
      const int k = s / p.S, e = s % p.S, KM = p.n_models * out;
      const size_t wc = (size_t)e * inp * KM;
      p.WT0cf[wc + (size_t)i * KM + (size_t)k * out + o] = v;
      p.WT0cq[wc + frag_off<bf16_t>(i, k * out + o, KM)] = f2bf(v);
    }
  } else {
    if (t >= in) return;
    p.wout[(size_t)s * in + t] = src[t];
    if (t == 0) p.bout[s] = src[in];
  }
}

void launch_pack(const PackArgs& p, int slots, hipStream_t st) {
  long maxel = 0;
  for (int l = 0; l < kLayers; ++l) {
    const long inp = l == 0 ? p.Fp : p.width[l];
    const long el = (long)p.width[l + 1] * inp;
    maxel = el > maxel ? el : maxel;
  }
  dim3 grid((unsigned)((maxel + 255) / 256), kLayers, slots);
  hipLaunchKernelGGL(k_pack, grid, dim3(256), 0, st, p);
}

}  // namespace nnp

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

template <typename T, int WM, int WN, int TM, int TN, int EPI, bool RESIDENT>
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
      const int r = idx / VPR, k = c * KC + (idx % VPR) * (16 / (int)sizeof(T));
      const unsigned off = k < K ? (unsigned)((r * a.lda + k) * (int)sizeof(T)) : kOutOfRange;
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

  const int ns = K / Frag<T>::KS;
  const int nchunks = (ns + SPC - 1) / SPC;  // RESIDENT: nchunks <= kMaxResident
  const int npass = a.N / NP;
  const int arow = (wm * TM * 16 + (lane & 15)) * kChunkStride + (lane >> 4) * 16;
  const int rl = lane & 15, cq = (lane >> 4) * 4;
  const float* bias = a.bias ? a.bias + (size_t)s * a.sBias : nullptr;
  const float ia = 1.f / a.alpha;
  unsigned char* stg = smem + (RESIDENT ? nchunks : 2) * BM * kChunkStride + wv * 16 * SS;
  const int col_w = wn * TN * 16;  // this wave's first column inside a pass

  f32x4_t acc[TM][TN];
  zero_acc(acc);
  BRing<T, TN, P> br;
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
  const int nk = (K + BK - 1) / BK;

  uint4 ra[NVA], rb[NVB];
  auto gload = [&](int kt) {
    const int k0 = kt * BK;
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

  gload(0);
  lstore(0);
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
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) Mfma<T>::mma(fa[i], fb[j], acc[i][j]);
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
// The rows of each element are cut into chunks of `chunk` rows; block
// (chunk, o-tile, i-tile) writes its partial sums, and a second kernel adds
// the partials of each element in chunk order (deterministic).

template <typename TD, typename TH>
__global__ __launch_bounds__(256) void k_wgrad(const GroupTable* __restrict__ gt, int S,
                                               const TD* __restrict__ D, int ldd, int Nout,
                                               const TH* __restrict__ H, int ldh, int Nin,
                                               int chunk, float* __restrict__ partial) {
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
      sh[rr][cc] = (ok && i0 + cc < Nin) ? Store<TH>::get(H + (size_t)row * ldh + i0 + cc) : 0.f;
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
  float* out = partial + (size_t)c * ((size_t)Nout * Nin + Nout);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int o = o0 + to + x, i = i0 + ti + y;
      if (o < Nout && i < Nin) out[(size_t)o * Nin + i] = acc[x][y];
    }
  if (blockIdx.z == 0 && tid < 64 && o0 + tid < Nout) out[(size_t)Nout * Nin + o0 + tid] = bacc;
}

// The same partials on MFMA (layers whose width is at least 16): the chunk's
// product dW = D^T H as C[i][o] = sum_r H[r][i] D[r][o], K = the chunk's
// rows.  One workgroup per (chunk, 128 o, 128 i) tile, four waves of 64 x 64
// (4 x 4 MFMA tiles).  Every stage reads BK rows of D and H with coalesced
// loads (16 or 32 lanes per 256- or 512-byte row segment) while the previous
// stage computes.
//   FP32 (v_mfma_f32_16x16x4f32, one K element per lane): the rows stay
//   row-major in LDS (144 floats per row, so the four K rows of a fragment
//   fall in different banks), and a fragment is one 4-byte read per lane.
//   BF16 (v_mfma_f32_16x16x32_bf16, eight consecutive K per lane): the tile is
//   transposed on its way into LDS, one LDS row per output (or input) holding
//   the stage's 64 atom rows, with the 16-byte granules of row c XOR-swizzled
//   by (c / 8) % 8 and rows 160 bytes apart; lanes 16 apart hold atom rows r
//   and r ^ 1 and swap them, so each 4-byte store writes an (r, r + 1) pair.
//   Stores then meet at most two to a bank and the 16-byte fragment reads
//   none (a CPU model of the layout checks every fragment).
// The i-tile-0 workgroups also sum db from the staged D.  The accumulator
// layout leaves each lane four consecutive i of one o, stored as one vector.
constexpr int kWgBO = 128, kWgBI = 128;

template <typename T> struct WgLayout;
template <> struct WgLayout<bf16_t> {
  static constexpr int BK = 64;                 // atom rows per stage
  static constexpr int P = 80;                  // elements per LDS row (160 bytes)
  static constexpr int TILE = 128 * P;          // elements per operand tile
  static constexpr int ITEMS = BK * 16 / 256;   // 16-byte loads per thread and operand
  __device__ __forceinline__ static int off(int c, int k) {
    return c * P + 8 * ((k >> 3) ^ ((c >> 3) & 7)) + (k & 7);
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

template <typename T>
__global__ __launch_bounds__(256) void k_wgrad_mfma(const GroupTable* __restrict__ gt, int S,
                                                    const T* __restrict__ D, int ldd, int Nout,
                                                    const T* __restrict__ H, int ldh, int Nin,
                                                    int chunk, float* __restrict__ partial) {
  using L = WgLayout<T>;
  constexpr bool BF = sizeof(T) == 2;
  constexpr int BK = L::BK, ITEMS = L::ITEMS;
  constexpr int CPL = 16 / sizeof(T);       // columns per 16-byte load
  constexpr int LPR = 128 / CPL;            // loads per 128-column row segment
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);

  const int c = blockIdx.x;
  if (c >= gt->n_wchunks) return;
  int s = 0;
  for (int q = 1; q < S; ++q) s = (c >= gt->wchunk[q]) ? q : s;
  const int r0 = gt->pstart[s] + (c - gt->wchunk[s]) * chunk;
  const int rend = gt->pstart[s] + gt->cnt[s];
  const int r1 = r0 + chunk < rend ? r0 + chunk : rend;
  const int o0 = blockIdx.y * kWgBO, i0 = blockIdx.z * kWgBI;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wo = w >> 1, wi = w & 1;  // this wave's 64 x 64 tile

  uint4 rd[ITEMS], rh[ITEMS];
  // item k of this thread: atom row f / LPR of the stage, column group f % LPR
  auto gload = [&](int rb) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int f = tid + 256 * k, r = f / LPR, g = f % LPR;
      const int row = rb + r;
      const bool rok = row < r1;
      const int oc = o0 + g * CPL, ic = i0 + g * CPL;
      rd[k] = rok && oc < Nout ? *reinterpret_cast<const uint4*>(D + (size_t)row * ldd + oc)
                               : make_uint4(0u, 0u, 0u, 0u);
      rh[k] = rok && ic < Nin ? *reinterpret_cast<const uint4*>(H + (size_t)row * ldh + ic)
                              : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto lstore = [&](int buf) __attribute__((always_inline)) {
    T* dt = lds + (size_t)buf * 2 * L::TILE;
    T* ht = dt + L::TILE;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int f = tid + 256 * k, r = f / LPR, g = f % LPR;
      if constexpr (BF) {
        // lanes 16 apart hold rows r and r ^ 1 of the same columns
        uint4 od, oh;
        od.x = __shfl_xor(rd[k].x, 16, 64); od.y = __shfl_xor(rd[k].y, 16, 64);
        od.z = __shfl_xor(rd[k].z, 16, 64); od.w = __shfl_xor(rd[k].w, 16, 64);
        oh.x = __shfl_xor(rh[k].x, 16, 64); oh.y = __shfl_xor(rh[k].y, 16, 64);
        oh.z = __shfl_xor(rh[k].z, 16, 64); oh.w = __shfl_xor(rh[k].w, 16, 64);
        const bool odd = r & 1;
        // even rows write columns 0..3 of the group, odd rows columns 4..7;
        // lo = the even row's element, hi = the odd row's
        const unsigned md[4] = {rd[k].x, rd[k].y, rd[k].z, rd[k].w};
        const unsigned pd[4] = {od.x, od.y, od.z, od.w};
        const unsigned mh[4] = {rh[k].x, rh[k].y, rh[k].z, rh[k].w};
        const unsigned ph[4] = {oh.x, oh.y, oh.z, oh.w};
        const int kr = r & ~1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int col = g * 8 + e + (odd ? 4 : 0);
          const int wd = (e + (odd ? 4 : 0)) >> 1;  // dword of the element
          const bool hi = (e & 1);                 // which half of it
          const unsigned ev_d = odd ? pd[wd] : md[wd], od_d = odd ? md[wd] : pd[wd];
          const unsigned ev_h = odd ? ph[wd] : mh[wd], od_h = odd ? mh[wd] : ph[wd];
          const unsigned vd = hi ? ((ev_d >> 16) | (od_d & 0xffff0000u))
                                 : ((ev_d & 0xffffu) | (od_d << 16));
          const unsigned vh = hi ? ((ev_h >> 16) | (od_h & 0xffff0000u))
                                 : ((ev_h & 0xffffu) | (od_h << 16));
          *reinterpret_cast<unsigned*>(dt + L::off(col, kr)) = vd;
          *reinterpret_cast<unsigned*>(ht + L::off(col, kr)) = vh;
        }
      } else {
        *reinterpret_cast<uint4*>(dt + r * L::RS + g * 4) = rd[k];
        *reinterpret_cast<uint4*>(ht + r * L::RS + g * 4) = rh[k];
      }
    }
  };

  f32x4_t acc[4][4];
  zero_acc(acc);
  float bacc = 0.f;
  const int nst = (r1 - r0 + BK - 1) / BK;
  if (nst > 0) {
    gload(r0);
    lstore(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) gload(r0 + (st + 1) * BK);
    const T* dt = lds + (size_t)buf * 2 * L::TILE;
    const T* ht = dt + L::TILE;
    if constexpr (BF) {
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const int j = kk * 4 + (lane >> 4);  // this lane's 8-row granule
        uint4 fa[4], fb[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int ci = wi * 64 + x * 16 + (lane & 15);
          fa[x] = *reinterpret_cast<const uint4*>(ht + ci * L::P + 8 * (j ^ ((ci >> 3) & 7)));
        }
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int co = wo * 64 + y * 16 + (lane & 15);
          fb[y] = *reinterpret_cast<const uint4*>(dt + co * L::P + 8 * (j ^ ((co >> 3) & 7)));
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) Mfma<bf16_t>::mma(fa[x], fb[y], acc[x][y]);
      }
      if (blockIdx.z == 0 && tid < kWgBO) {
        for (int k = 0; k < BK; ++k) bacc += bf2f(dt[L::off(tid, k)]);
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
      if (blockIdx.z == 0 && tid < kWgBO) {
        for (int k = 0; k < BK; ++k) bacc += dt[k * L::RS + tid];
      }
    }
    if (st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }
  // acc[x][y][e]: i = i0 + wi 64 + x 16 + 4 (lane / 16) + e, o = o0 + wo 64 + y 16 + lane % 16
  float* out = partial + (size_t)c * ((size_t)Nout * Nin + Nout);
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
  if (blockIdx.z == 0 && tid < kWgBO && o0 + tid < Nout) out[(size_t)Nout * Nin + o0 + tid] = bacc;
}

// out[s] (W then b, Nout*Nin + Nout floats at param_off[s]) = sum of partials.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const GroupTable* __restrict__ gt, int S,
                                                      const float* __restrict__ partial, int len,
                                                      float* __restrict__ dparams,
                                                      const long* __restrict__ param_off) {
  const int s = blockIdx.y;
  if (s >= S) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  float v = 0.f;
  for (int c = gt->wchunk[s]; c < gt->wchunk[s + 1]; ++c) v += partial[(size_t)c * len + e];
  dparams[param_off[s] + e] = v;
}

template <typename TD, typename TH>
void launch_wgrad(const GroupTable* gt, int S, int n_chunks_cap, const TD* D, int ldd, int Nout,
                  const TH* H, int ldh, int Nin, int chunk, float* partial, float* dparams,
                  const long* param_off_dev, hipStream_t st) {
  if constexpr (std::is_same<TD, TH>::value) {
    if (Nout >= 16 && Nout % 4 == 0 && Nin % 4 == 0 && ldd % 8 == 0 && ldh % 8 == 0) {
      static const bool attr = (ensure_lds(k_wgrad_mfma<TD>), true);
      (void)attr;
      dim3 grid(n_chunks_cap, (Nout + kWgBO - 1) / kWgBO, (Nin + kWgBI - 1) / kWgBI);
      hipLaunchKernelGGL(k_wgrad_mfma<TD>, grid, dim3(256), wgrad_lds_bytes<TD>(), st, gt, S, D,
                         ldd, Nout, H, ldh, Nin, chunk, partial);
      const int len = Nout * Nin + Nout;
      hipLaunchKernelGGL(k_wgrad_reduce, dim3((len + 255) / 256, S), dim3(256), 0, st, gt, S,
                         partial, len, dparams, param_off_dev);
      return;
    }
  }
  dim3 grid(n_chunks_cap, (Nout + 63) / 64, (Nin + 63) / 64);
  hipLaunchKernelGGL((k_wgrad<TD, TH>), grid, dim3(256), 0, st, gt, S, D, ldd, Nout, H, ldh, Nin,
                     chunk, partial);
  const int len = Nout * Nin + Nout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((len + 255) / 256, S), dim3(256), 0, st, gt, S, partial,
                     len, dparams, param_off_dev);
}
template void launch_wgrad<float, float>(const GroupTable*, int, int, const float*, int, int,
                                         const float*, int, int, int, float*, float*, const long*,
                                         hipStream_t);
template void launch_wgrad<bf16_t, bf16_t>(const GroupTable*, int, int, const bf16_t*, int, int,
                                           const bf16_t*, int, int, int, float*, float*,
                                           const long*, hipStream_t);
template void launch_wgrad<float, bf16_t>(const GroupTable*, int, int, const float*, int, int,
                                          const bf16_t*, int, int, int, float*, float*,
                                          const long*, hipStream_t);

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
    const float v = i < in ? src[(size_t)o * in + i] : 0.f;
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

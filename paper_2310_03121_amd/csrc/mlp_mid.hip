// Fused middle of the per-element networks (BF16 operands, FP32 accumulate):
// layer 2, the energy head, and the adjoint of layers 3 and 2, for one tile of
// 64 species-sorted rows per workgroup.
//
//   H2 = CELU(H1 W1^T + b1)                       (kept in LDS)
//   z3 = H2 W2^T + b2;  E_i = w_out . CELU(z3) + b_out
//   D3 = up_i * w_out * CELU'(z3)                 (kept in LDS)
//   D2 = (D3 W2) * CELU'(z2)                      (written over H2 in LDS)
//   D1 = (D2 W1) * CELU'(z1)                      (to global)
//
// CELU'(z) is recovered from the stored activation: 1 for h > 0, else
// 1 + h/alpha.  The four products are MFMA GEMMs with the A operand resident
// in LDS and the weight operand streamed through a double-buffered LDS stage
// of 64 K-columns.  This removes three launches and the HBM round trips of
// H2, D3 and D2 that separate layer kernels would need.  Optional pointers
// also store H2, H3, D3 and D2 for the parameter gradients.
#include "kernels.h"

namespace nnp {

typedef __bf16 bf16x8_mid __attribute__((ext_vector_type(8)));
typedef float floatx4_mid __attribute__((ext_vector_type(4)));

constexpr int kMidBM = 64;
constexpr int kMidBK = 64;
constexpr int kMidBS = kMidBK + 8;  // LDS stride of a staged weight row (elements)

__device__ __forceinline__ int rup64(int x) { return (x + 63) / 64 * 64; }

// C[64 x N] = A[64 x K] (LDS, stride sa) * B[N x K]^T (global, stride ldb).
// Waves 2 x 2: wave (wm, wn) owns rows wm*32 .. +31 and columns wn*16*TN .. .
template <int TN>
__device__ __forceinline__ void mid_gemm(const bf16_t* As, int sa, const bf16_t* __restrict__ Bg,
                                         int ldb, int N, int K, bf16_t* Bs,
                                         floatx4_mid (&acc)[2][TN], int tid, int lane, int wm,
                                         int wn) {
  constexpr int NVB = (2 * 16 * TN * 8 + 255) / 256;  // 16-byte vectors per thread per stage
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4_mid{0.f, 0.f, 0.f, 0.f};
  const int nk = (K + kMidBK - 1) / kMidBK;
  uint4 rb[NVB];
  auto gload = [&](int kt) {
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx >> 3, sg = idx & 7;
      const int k = kt * kMidBK + sg * 8;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (r < N && k < K) val = *reinterpret_cast<const uint4*>(Bg + (size_t)r * ldb + k);
      rb[v] = val;
    }
  };
  auto lstore = [&](int buf) {
    bf16_t* bs = Bs + buf * 256 * kMidBS;
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const int idx = tid + v * 256;
      const int r = idx >> 3, sg = idx & 7;
      if (r < N) *reinterpret_cast<uint4*>(bs + r * kMidBS + sg * 8) = rb[v];
    }
  };
  gload(0);
  lstore(0);
  __syncthreads();
  const int rl = lane & 15, kq = (lane >> 4) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    const bf16_t* bs = Bs + buf * 256 * kMidBS + (wn * 16 * TN + rl) * kMidBS + kq;
    const bf16_t* as = As + (wm * 32 + rl) * sa + kt * kMidBK + kq;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      uint4 fa[2], fb[TN];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        fa[i] = *reinterpret_cast<const uint4*>(as + i * 16 * sa + kk * 32);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        fb[j] = *reinterpret_cast<const uint4*>(bs + j * 16 * kMidBS + kk * 32);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8_mid, fa[i]), __builtin_bit_cast(bf16x8_mid, fb[j]),
              acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) lstore(buf ^ 1);
    __syncthreads();
  }
}

__device__ __forceinline__ float celu_mid(float z, float alpha, float inv_alpha_l2e) {
  return z > 0.f ? z : alpha * (__builtin_amdgcn_exp2f(z * inv_alpha_l2e) - 1.f);
}

__device__ __forceinline__ float dcelu_from_h(float h, float inv_alpha) {
  return h > 0.f ? 1.f : 1.f + h * inv_alpha;
}

template <int W1, int W2, int W3>
__global__ __launch_bounds__(256) void k_mlp_mid(MidArgs a) {
  constexpr int TA = W2 / 32, TB = W3 / 32, TC = W2 / 32, TD = W1 / 32;
  constexpr int S1 = (W1 + 63) / 64 * 64 + 8;  // LDS strides (elements)
  constexpr int S2 = (W2 + 63) / 64 * 64 + 8;
  constexpr int S3 = (W3 + 63) / 64 * 64 + 8;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  bf16_t* L1 = reinterpret_cast<bf16_t*>(smem);  // H1 tile
  bf16_t* L2 = L1 + kMidBM * S1;                  // H2, then D2
  bf16_t* L3 = L2 + kMidBM * S2;                  // D3
  bf16_t* Bs = L3 + kMidBM * S3;                  // weight stages
  float* epart = reinterpret_cast<float*>(Bs + 2 * 256 * kMidBS);  // [2][64]

  const GroupTable* gt = a.gt;
  const int row0 = blockIdx.x * kMidBM;
  if (row0 >= gt->total_rows) return;
  int s = 0;
#pragma unroll
  for (int q = 1; q < kMaxS; ++q) s = (row0 >= gt->pstart[q]) ? q : s;
  const int row_end = gt->pstart[s] + gt->cnt[s];
  if (row0 >= row_end) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int rl = lane & 15, rq = (lane >> 4) * 4;
  const float alpha = a.alpha, ia = 1.f / a.alpha, ial2e = a.inv_alpha_l2e;

  // H1 tile -> LDS (zero rows past the group, zero K padding)
  for (int idx = tid; idx < kMidBM * (S1 - 8) / 8; idx += 256) {
    const int r = idx / ((S1 - 8) / 8), c = (idx % ((S1 - 8) / 8)) * 8;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (row0 + r < row_end && c < W1)
      v = *reinterpret_cast<const uint4*>(a.H1 + (size_t)(row0 + r) * W1 + c);
    *reinterpret_cast<uint4*>(L1 + r * S1 + c) = v;
  }
  // zero the K padding of the H2/D2 and D3 regions (read as A operands)
  constexpr int P2 = (S2 - 8) - W2, P3 = (S3 - 8) - W3;
  if constexpr (P3 > 0)
    for (int idx = tid; idx < kMidBM * P3; idx += 256) L3[(idx / P3) * S3 + W3 + idx % P3] = 0;
  if constexpr (P2 > 0)
    for (int idx = tid; idx < kMidBM * P2; idx += 256) L2[(idx / P2) * S2 + W2 + idx % P2] = 0;
  __syncthreads();

  // ---- H2 = CELU(H1 W1^T + b1)
  {
    floatx4_mid acc[2][TA];
    mid_gemm<TA>(L1, S1, a.W1 + (size_t)s * W2 * W1, W1, W2, W1, Bs, acc, tid, lane, wm, wn);
    const float* b1 = a.b1 + (size_t)s * W2;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wm * 32 + i * 16 + rq + e;
        const bool rv = row0 + r < row_end;
#pragma unroll
        for (int j = 0; j < TA; ++j) {
          const int c = wn * 16 * TA + j * 16 + rl;
          const float h = rv ? celu_mid(acc[i][j][e] + b1[c], alpha, ial2e) : 0.f;
          L2[r * S2 + c] = f2bf(h);
          if (a.H2) a.H2[(size_t)(row0 + r) * W2 + c] = f2bf(h);
        }
      }
  }
  __syncthreads();

  // ---- z3 = H2 W2^T + b2: energies and D3
  {
    floatx4_mid acc[2][TB];
    mid_gemm<TB>(L2, S2, a.W2 + (size_t)s * W3 * W2, W2, W3, W2, Bs, acc, tid, lane, wm, wn);
    const float* b2 = a.b2 + (size_t)s * W3;
    const float* wo = a.wout + (size_t)s * W3;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wm * 32 + i * 16 + rq + e;
        const int row = row0 + r;
        const bool rv = row < row_end;
        float up = 0.f;
        if (rv) up = a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f;
        float ep = 0.f;
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const int c = wn * 16 * TB + j * 16 + rl;
          const float z = acc[i][j][e] + b2[c];
          const float ex = __builtin_amdgcn_exp2f(fminf(z, 0.f) * ial2e);
          const float h = z > 0.f ? z : alpha * (ex - 1.f);
          const float d = rv ? up * wo[c] * (z > 0.f ? 1.f : ex) : 0.f;
          ep += rv ? wo[c] * h : 0.f;
          L3[r * S3 + c] = f2bf(d);
          if (a.H3) a.H3[(size_t)row * W3 + c] = f2bf(rv ? h : 0.f);
          if (a.D3) a.D3[(size_t)row * W3 + c] = f2bf(d);
        }
        ep += __shfl_xor(ep, 1, 64);
        ep += __shfl_xor(ep, 2, 64);
        ep += __shfl_xor(ep, 4, 64);
        ep += __shfl_xor(ep, 8, 64);
        if (rl == 0) epart[wn * kMidBM + r] = ep;
      }
  }
  __syncthreads();
  if (tid < kMidBM) {
    const int row = row0 + tid;
    if (row < row_end) a.erow[row] = epart[tid] + epart[kMidBM + tid] + a.bout[s];
    if (a.uprow) {
      float up = 0.f;
      if (row < row_end) up = a.dLdE ? (float)a.dLdE[a.mol[a.perm[row]]] : 1.f;
      a.uprow[row] = up;
    }
  }

  // ---- D2 = (D3 W2) * CELU'(z2), written over H2
  {
    floatx4_mid acc[2][TC];
    mid_gemm<TC>(L3, S3, a.W2T + (size_t)s * W2 * W3, W3, W2, W3, Bs, acc, tid, lane, wm, wn);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wm * 32 + i * 16 + rq + e;
        const bool rv = row0 + r < row_end;
#pragma unroll
        for (int j = 0; j < TC; ++j) {
          const int c = wn * 16 * TC + j * 16 + rl;
          const float h = bf2f(L2[r * S2 + c]);
          const float d = rv ? acc[i][j][e] * dcelu_from_h(h, ia) : 0.f;
          L2[r * S2 + c] = f2bf(d);
          if (a.D2) a.D2[(size_t)(row0 + r) * W2 + c] = f2bf(d);
        }
      }
  }
  __syncthreads();

  // ---- D1 = (D2 W1) * CELU'(z1) -> global
  {
    floatx4_mid acc[2][TD];
    mid_gemm<TD>(L2, S2, a.W1T + (size_t)s * W1 * W2, W2, W1, W2, Bs, acc, tid, lane, wm, wn);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = wm * 32 + i * 16 + rq + e;
        const bool rv = row0 + r < row_end;
#pragma unroll
        for (int j = 0; j < TD; ++j) {
          const int c = wn * 16 * TD + j * 16 + rl;
          const float h = bf2f(L1[r * S1 + c]);
          const float d = rv ? acc[i][j][e] * dcelu_from_h(h, ia) : 0.f;
          a.D1[(size_t)(row0 + r) * W1 + c] = f2bf(d);
        }
      }
  }
}

template <int W1, int W2, int W3>
static size_t mid_lds() {
  constexpr int S1 = (W1 + 63) / 64 * 64 + 8, S2 = (W2 + 63) / 64 * 64 + 8,
                S3 = (W3 + 63) / 64 * 64 + 8;
  return (size_t)2 * (kMidBM * (S1 + S2 + S3) + 2 * 256 * kMidBS) + 2 * kMidBM * 4;
}

template <int W1, int W2, int W3>
static void launch_mid_t(const MidArgs& a, int rows_cap, hipStream_t st) {
  const size_t lds = mid_lds<W1, W2, W3>();
  static const bool attr = (ensure_lds(k_mlp_mid<W1, W2, W3>), true);
  (void)attr;
  hipLaunchKernelGGL((k_mlp_mid<W1, W2, W3>), dim3((rows_cap + kMidBM - 1) / kMidBM), dim3(256),
                     lds, st, a);
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

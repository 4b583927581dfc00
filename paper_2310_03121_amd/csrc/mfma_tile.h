// MFMA building blocks shared by the network kernels.
//
// A wave owns a (TM*16) x (TN*16) block of C = A * B^T.  The activations A
// sit in LDS (row-major, a byte stride per row); the weights B ([N][K]
// row-major, the same for every row tile of an element and therefore L2
// resident) are read from global memory straight into MFMA operand registers,
// P k-steps ahead of their use, so weights need neither LDS space nor
// barriers.  The MFMA is issued with the operands swapped (B as the first
// source), which leaves each lane holding four consecutive columns of one row
// of C: lane l has row l % 16 and columns 4 * (l / 16) + {0, 1, 2, 3} of each
// 16 x 16 tile, so epilogues store 4-column vectors.
//
// Fragment of a k-step (16 bytes per lane, BF16): lane l holds row l % 16 of
// its 16-row slice, elements [8 * (l / 16), +8) of the k-step's 32 (one
// v_mfma_f32_16x16x32_bf16).  A is read that way from row-major LDS; B is
// pre-packed so that the 64 lanes' fragments are contiguous.
#pragma once
#include "kernels.h"

namespace nnp {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

// Word 3 of a raw buffer resource on CDNA (32-bit data format, no swizzle):
// buffer loads whose offset lies past the resource's byte range return zero.
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr unsigned kOutOfRange = 0x80000000u;

template <typename T> struct Frag;
template <> struct Frag<bf16_t> {
  static constexpr int KS = 32;  // K per k-step
  static constexpr int EL = 8;   // elements per lane per fragment
  __device__ __forceinline__ static void mma(const uint4& b, const uint4& a, f32x4_t& acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, b),
                                                  __builtin_bit_cast(bf16x8_t, a), acc, 0, 0, 0);
  }
};

// Register ring of weight fragments: slot u holds the TN fragments of every
// k-step s with s % P == u.  Loads are unconditional (a step past the end
// re-reads the last step, which keeps every access inside B), so the wait
// before a step's MFMAs is an exact count of the loads issued after it.
// B is stored in fragment order (see k_pack): tile nt, k-step ks, lane l at
// ((nt * (K/KS) + ks) * 64 + l) * EL, so each fragment load is one contiguous
// 1 KB block per wave.  Steps are counted per pass over [0, nsp), nsp = ns
// rounded up to the ring depth: steps in [ns, nsp) re-read the last step
// (their A columns are zero), and steps from nsp on read the next pass's
// steps, so a pass's first fragments arrive while the previous one ends.
template <typename T, int TN, int P>
struct BRing {
  static constexpr int FE = 64 * Frag<T>::EL;  // elements per fragment
  uint4 r[P][TN];
  const T* base;       // this pass: fragment (n_first / 16, 0) + this lane
  const T* base_next;  // next pass (or this one again after the last)
  size_t tile;         // elements per 16-row tile (all k-steps)
  int ns, nsp;
  __device__ __forceinline__ const T* at(const T* B, int n_first, int lane) const {
    return B + (size_t)(n_first / 16) * tile + lane * Frag<T>::EL;
  }
  __device__ __forceinline__ void init(const T* B, int n_first, int n_next, int lane, int K) {
    ns = K / Frag<T>::KS;
    nsp = (ns + P - 1) / P * P;
    tile = (size_t)ns * FE;
    base = at(B, n_first, lane);
    base_next = n_next >= 0 ? at(B, n_next, lane) : base;
  }
  __device__ __forceinline__ void next_pass(const T* B, int n_next, int lane) {
    base = base_next;
    base_next = n_next >= 0 ? at(B, n_next, lane) : base;
  }
  template <int U>
  __device__ __forceinline__ void load(int s) {
    const T* p = s < ns ? base + (size_t)s * FE
                        : (s < nsp ? base + (size_t)(ns - 1) * FE : base_next + (size_t)(s - nsp) * FE);
#pragma unroll
    for (int j = 0; j < TN; ++j) r[U][j] = *reinterpret_cast<const uint4*>(p + j * tile);
  }
  template <int U = 0>
  __device__ __forceinline__ void prologue() {
    if constexpr (U < P) {
      load<U>(U);
      prologue<U + 1>();
    }
  }
};

// Lane l: the l-th set bit of m (0 when m has at most l set bits).
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int l) {
  int q = 0;
#pragma unroll
  for (int w = 32; w; w >>= 1) {
    const int t = q + w;
    if (__popcll(m & ((1ull << t) - 1ull)) <= l) q = t;
  }
  return l < __popcll(m) ? q : 0;
}

// A ring over a compacted list of k-steps: position s of the product is
// k-step `qlist` of lane s (qlist holds the tile's active k-steps in order,
// one per lane), so steps whose A columns are zero for the whole tile are
// never issued.  Positions from ns on re-read the last active step (k-step 0
// when there is none), which keeps every access inside B.
template <typename T, int TN, int P>
struct BRingQ {
  static constexpr int FE = 64 * Frag<T>::EL;
  uint4 r[P][TN];
  const T* base;  // fragment (n_first / 16, 0) + this lane
  size_t tile;
  int ns;         // active k-steps (uniform)
  int qlist;      // lane l: the k-step of position l
  __device__ __forceinline__ void init(const T* B, int n_first, int lane, int K, int ns_,
                                       int qlist_) {
    tile = (size_t)(K / Frag<T>::KS) * FE;
    base = B + (size_t)(n_first / 16) * tile + lane * Frag<T>::EL;
    ns = ns_;
    qlist = qlist_;
  }
  template <int U>
  __device__ __forceinline__ void load(int s) {
    const int pc = s < ns ? s : (ns > 0 ? ns - 1 : 0);
    const int q = __builtin_amdgcn_readlane(qlist, pc);
    const T* p = base + (size_t)q * FE;
#pragma unroll
    for (int j = 0; j < TN; ++j) r[U][j] = *reinterpret_cast<const uint4*>(p + j * tile);
  }
  template <int U = 0>
  __device__ __forceinline__ void prologue() {
    if constexpr (U < P) {
      load<U>(U);
      prologue<U + 1>();
    }
  }
  __device__ __forceinline__ void next_pass(const T*, int, int) {}  // one pass only
};

// A ring for a product whose four 16-column tiles come in two pairs at
// arbitrary places: tiles (2 c0, 2 c0 + 1, 2 c1, 2 c1 + 1) of B (K dense,
// ns = K / KS steps, a multiple of P).  Steps from ns on read the next
// pass's pair of pairs, as BRing does.
template <typename T, int P>
struct BRingPair {
  static constexpr int FE = 64 * Frag<T>::EL;
  uint4 r[P][4];
  const T* b0;
  const T* b1;   // this pass
  const T* n0;
  const T* n1;   // the next one
  size_t tile;
  int ns;
  __device__ __forceinline__ const T* at(const T* B, int c, int lane) const {
    return B + (size_t)(2 * c) * tile + lane * Frag<T>::EL;
  }
  __device__ __forceinline__ void init(const T* B, int K, int lane, int c0, int c1, int d0,
                                       int d1) {
    ns = K / Frag<T>::KS;
    tile = (size_t)ns * FE;
    b0 = at(B, c0, lane);
    b1 = at(B, c1, lane);
    n0 = at(B, d0, lane);
    n1 = at(B, d1, lane);
  }
  __device__ __forceinline__ void next_pass(const T* B, int d0, int d1, int lane) {
    b0 = n0;
    b1 = n1;
    n0 = at(B, d0, lane);
    n1 = at(B, d1, lane);
  }
  template <int U>
  __device__ __forceinline__ void load(int s) {
    const T* p0 = s < ns ? b0 + (size_t)s * FE : n0 + (size_t)(s - ns) * FE;
    const T* p1 = s < ns ? b1 + (size_t)s * FE : n1 + (size_t)(s - ns) * FE;
    r[U][0] = *reinterpret_cast<const uint4*>(p0);
    r[U][1] = *reinterpret_cast<const uint4*>(p0 + tile);
    r[U][2] = *reinterpret_cast<const uint4*>(p1);
    r[U][3] = *reinterpret_cast<const uint4*>(p1 + tile);
  }
  template <int U = 0>
  __device__ __forceinline__ void prologue() {
    if constexpr (U < P) {
      load<U>(U);
      prologue<U + 1>();
    }
  }
};

template <int TM>
__device__ __forceinline__ void load_a(const unsigned char* arow, int astride16, uint4 (&fa)[TM]) {
#pragma unroll
  for (int i = 0; i < TM; ++i) fa[i] = *reinterpret_cast<const uint4*>(arow + i * astride16);
}

// One k-step: TM x TN MFMAs of the A fragments `fa` (already in registers)
// against ring slot U; if PREF, the next step's A fragments (at `anext`) are
// read from LDS into `fn` first, so their latency hides behind these MFMAs;
// then (if REFILL) the slot is refilled with step s_next.  The scheduling
// barrier keeps the refill right behind the step: left alone, the compiler
// sinks all refills of a group to its end, which removes the prefetch.
template <typename T, int TM, int TN, int P, int U, bool REFILL, bool PREF, typename Ring>
__device__ __forceinline__ void kstep(const unsigned char* anext, int astride16,
                                      Ring& br, int s_next, f32x4_t (&acc)[TM][TN],
                                      const uint4 (&fa)[TM], uint4 (&fn)[TM]) {
  if constexpr (PREF) load_a<TM>(anext, astride16, fn);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) Frag<T>::mma(br.r[U][j], fa[i], acc[i][j]);
  if constexpr (REFILL) br.template load<U>(s_next);
  __builtin_amdgcn_sched_barrier(0);
}

// A group of P consecutive k-steps s0 .. s0+P-1 (s0 a multiple of P), A
// starting at `ap` for step s0; every step refills its slot with step + P.
template <typename T, int TM, int TN, int P, typename Ring>
__device__ __forceinline__ void kgroup(const unsigned char* ap, int astride16, Ring& br,
                                       int s0, f32x4_t (&acc)[TM][TN]) {
  static_assert(P == 4, "four steps per group");
  constexpr int SB = Frag<T>::KS * sizeof(T);
  uint4 f0[TM], f1[TM];
  load_a<TM>(ap, astride16, f0);
  kstep<T, TM, TN, P, 0, true, true>(ap + SB, astride16, br, s0 + P, acc, f0, f1);
  kstep<T, TM, TN, P, 1, true, true>(ap + 2 * SB, astride16, br, s0 + 1 + P, acc, f1, f0);
  kstep<T, TM, TN, P, 2, true, true>(ap + 3 * SB, astride16, br, s0 + 2 + P, acc, f0, f1);
  kstep<T, TM, TN, P, 3, true, false>(ap, astride16, br, s0 + 3 + P, acc, f1, f0);
}

// All NS k-steps of a product with compile-time K, fully unrolled: slot
// refills stop at the last step, so no load is wasted.  The two A fragment
// sets alternate by step parity.
template <typename T, int TM, int TN, int P, int NS, int S = 0>
__device__ __forceinline__ void ksteps_ct(const unsigned char* a0, int astride16,
                                          BRing<T, TN, P>& br, f32x4_t (&acc)[TM][TN],
                                          uint4 (&fe)[TM], uint4 (&fo)[TM]) {
  if constexpr (S < NS) {
    constexpr int SB = Frag<T>::KS * sizeof(T);
    if constexpr (S == 0) load_a<TM>(a0, astride16, fe);
    if constexpr (S % 2 == 0)
      kstep<T, TM, TN, P, S % P, (S + P < NS), (S + 1 < NS)>(a0 + (S + 1) * SB, astride16, br,
                                                             S + P, acc, fe, fo);
    else
      kstep<T, TM, TN, P, S % P, (S + P < NS), (S + 1 < NS)>(a0 + (S + 1) * SB, astride16, br,
                                                             S + P, acc, fo, fe);
    ksteps_ct<T, TM, TN, P, NS, S + 1>(a0, astride16, br, acc, fe, fo);
  }
}

template <int TM, int TN>
__device__ __forceinline__ void zero_acc(f32x4_t (&acc)[TM][TN]) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
}

// Workgroup b of nb -> row tile, so that the tiles of one XCD (dispatch goes
// round-robin over the eight XCDs) are consecutive: neighbouring tiles share
// an element and hence the weights their XCD's L2 holds.  nb must be the
// number of tiles that hold rows (not the grid size): every XCD then gets
// its share of real tiles, and blocks b >= nb exit.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Species of the tile starting at row0 (groups start at multiples of kPad).
__device__ __forceinline__ int tile_species(const GroupTable* gt, int row0) {
  int s = 0;
#pragma unroll
  for (int q = 1; q < kMaxS; ++q) s = (row0 >= gt->pstart[q]) ? q : s;
  return s;
}

__device__ __forceinline__ float celu_fwd(float z, float alpha, float inv_alpha_l2e) {
  return z > 0.f ? z : alpha * (__builtin_amdgcn_exp2f(z * inv_alpha_l2e) - 1.f);
}

__device__ __forceinline__ float celu_slope(float h, float inv_alpha) {
  return h > 0.f ? 1.f : 1.f + h * inv_alpha;
}

template <typename T> struct Vec4;
template <> struct Vec4<float> {
  __device__ __forceinline__ static float4 get(const float* p) {
    return *reinterpret_cast<const float4*>(p);
  }
};
template <> struct Vec4<bf16_t> {
  __device__ __forceinline__ static float4 get(const bf16_t* p) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
};

}  // namespace nnp

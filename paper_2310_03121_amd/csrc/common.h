// Shared device-side definitions of the NNP engine (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnp {

constexpr int kWave = 64;
constexpr int kNR = 16;       // radial shifts per species block
constexpr int kNA = 4;        // angular radial shifts
constexpr int kNZ = 8;        // angle shifts
constexpr int kMaxS = 8;      // species supported
constexpr int kMaxModels = 8; // ensemble members supported
constexpr int kPad = 128;     // species groups start at multiples of this row count
constexpr int kLayers = 4;    // Linear layers per element network

// Device status bits (workspace word 0).
enum : uint32_t {
  kStSpecies = 1u << 0,
  kStNonFinite = 1u << 1,
  kStCapacity = 1u << 2,
  kStOffsets = 1u << 3,
};

// Symmetry-function constants, passed by value to the kernels.
struct AevConst {
  int S;             // species
  int F;             // features per atom
  int Fp;            // row stride of the feature matrix (A0 + angular columns, rounded up to 64)
  int A0;            // first angular column: S * 16 rounded up to 32, so that every
                     // angular block is one 32-column k-step of the network (the
                     // gap columns are zero; S * 16 for rows in the published order)
  float rc2_r;       // fl32(rc_r * rc_r): radial predicate
  float rc2_a;       // fl32(rc_a * rc_a): angular predicate
  float inv_rc_r;    // 1 / rc_r
  float inv_rc_a;    // 1 / rc_a
  float pi_2rc_r;    // pi / (2 rc_r): cutoff derivative scale
  float pi_2rc_a;
  float eta_r_l2e;   // eta_r * log2(e)
  float eta_r2;      // 2 * eta_r
  float eta_a_l2e;   // eta_a * log2(e)
  float eta_a;       // eta_a
  float zeta;
  float cR;          // radial prefactor
  float kappa;       // angle cosine scale
  float shf_r[kNR];
  float shf_a[kNA];
  float cos_z[kNZ];
  float sin_z[kNZ];
  // device copy of shf_r, cos_z, sin_z (kNR + 2 kNZ floats): per-lane
  // constants are one cached load each instead of a select chain
  const float* lane_tab;
};

// Periodic-box description.  periodic: 0 none, 1 orthorhombic (edges L),
// 2 triclinic (rows v[0] = a = (ax,0,0), v[1] = b = (bx,by,0),
// v[2] = c = (cx,cy,cz), reduced form; cells are binned in fractional
// coordinates).  nc[d] == 1 means that dimension is not binned (the box is
// too small for three cells).
struct BoxConst {
  int periodic;
  float L[3];
  float invL[3];
  int nc[3];
  float cell_scale[3];   // nc / L
  float v[3][3];         // triclinic cell rows
  float inv_diag[3];     // fl32(1 / v[d][d])
};

// Group table written by the species sort (device memory, int32):
//   cnt[0..7], pstart[0..8], wchunk_start[0..8], total_rows, n_wchunks
struct GroupTable {
  int cnt[kMaxS];
  int pstart[kMaxS + 1];
  int wchunk[kMaxS + 1];
  int total_rows;
  int n_wchunks;
  int pad[6];
};

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the wave, returned in every lane (all lanes active): inclusive
// prefix sums inside each row of 16 lanes by DPP row shifts (no LDS round
// trips), then the four row totals read from lanes 15, 31, 47 and 63.
__device__ __forceinline__ float wave_sum_rows(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));
  const int b = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_readlane(b, 15)) +
         __int_as_float(__builtin_amdgcn_readlane(b, 31)) +
         __int_as_float(__builtin_amdgcn_readlane(b, 47)) +
         __int_as_float(__builtin_amdgcn_readlane(b, 63));
}

// Butterfly sums over groups of 8 and 16 consecutive lanes by DPP (all
// lanes active), the same pairing as exchanges at lane distance 1, 2, 4 (and
// 8): swaps inside quads, then the half-row and row mirrors, which pair each
// lane with one of the other quad (half-row).  Every lane of a group gets the
// group's sum, with the same rounding in every lane.
template <int CTRL>
__device__ __forceinline__ float dpp_get(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float group8_sum(float v) {
  v += dpp_get<0xb1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_get<0x4e>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_get<0x141>(v);  // row_half_mirror
  return v;
}
__device__ __forceinline__ float group16_sum(float v) {
  v = group8_sum(v);
  v += dpp_get<0x140>(v);  // row_mirror
  return v;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Orders LDS traffic of the lanes of one wave (no cross-wave effect).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Lanes below this one whose bit is set in m.
__device__ __forceinline__ int popc_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// ------------------------------------------------------------- bf16 helpers

typedef uint16_t bf16_t;

// round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ bf16_t f2bf(float f) {
  return __builtin_bit_cast(bf16_t, (__bf16)f);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  const bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float bf2f(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <typename T> struct Store;
template <> struct Store<float> {
  __device__ __forceinline__ static void put(float* p, float v) { *p = v; }
  __device__ __forceinline__ static float get(const float* p) { return *p; }
  __device__ __forceinline__ static void put4(float* p, float4 v) {
    *reinterpret_cast<float4*>(p) = v;
  }
};
template <> struct Store<bf16_t> {
  __device__ __forceinline__ static void put(bf16_t* p, float v) { *p = f2bf(v); }
  __device__ __forceinline__ static float get(const bf16_t* p) { return bf2f(*p); }
  __device__ __forceinline__ static void put4(bf16_t* p, float4 v) {
    *reinterpret_cast<uint2*>(p) = make_uint2(f2bf2(v.x, v.y), f2bf2(v.z, v.w));
  }
};

// ------------------------------------------------------------- fp32 predicate

// Displacement component in float32 without contraction (minimum image when
// periodic), exactly as the neighbor predicate defines it.
__device__ __forceinline__ float disp(float xi, float xj, float L, float invL, int per) {
  float d = __fsub_rn(xj, xi);
  if (per) d = __fsub_rn(d, __fmul_rn(L, rintf(__fmul_rn(d, invL))));
  return d;
}

// Displacement in a reduced triclinic cell, float32 without contraction: the
// image is removed along c, then b, then a, n = rint(d_k / v_kk) each time.
// With the cutoff at most half of every perpendicular width this is the
// minimum image of every pair inside the cutoff.
__device__ __forceinline__ void tric_disp(float4 pi, float4 pj, const BoxConst& B, float& dx,
                                          float& dy, float& dz) {
  dx = __fsub_rn(pj.x, pi.x);
  dy = __fsub_rn(pj.y, pi.y);
  dz = __fsub_rn(pj.z, pi.z);
  float n = rintf(__fmul_rn(dz, B.inv_diag[2]));
  dx = __fsub_rn(dx, __fmul_rn(B.v[2][0], n));
  dy = __fsub_rn(dy, __fmul_rn(B.v[2][1], n));
  dz = __fsub_rn(dz, __fmul_rn(B.v[2][2], n));
  n = rintf(__fmul_rn(dy, B.inv_diag[1]));
  dx = __fsub_rn(dx, __fmul_rn(B.v[1][0], n));
  dy = __fsub_rn(dy, __fmul_rn(B.v[1][1], n));
  n = rintf(__fmul_rn(dx, B.inv_diag[0]));
  dx = __fsub_rn(dx, __fmul_rn(B.v[0][0], n));
}

__device__ __forceinline__ float dist2(float dx, float dy, float dz) {
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

__device__ __forceinline__ int species_of(float4 p) { return __float_as_int(p.w); }

// Raises a kernel's dynamic LDS limit to what the gfx950 maximum (160 KB per
// workgroup; the default is 64 KB) leaves beside the kernel's static LDS, once
// per kernel, before its first launch (so never while a stream is being
// captured into a graph).  A limit above that maximum would be rejected.
template <typename K>
inline void ensure_lds(K* kernel) {
  hipFuncAttributes fa{};
  size_t stat = 0;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) == hipSuccess)
    stat = fa.sharedSizeBytes;
  const size_t lim = 160 * 1024;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(stat < lim ? lim - stat : 0));
}

// Clamp a (possibly corrupt) index into [0, n).
__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

}  // namespace nnp

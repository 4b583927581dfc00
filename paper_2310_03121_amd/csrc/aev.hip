// Atomic environment vectors (forward) and their adjoint with the force
// scatter, one wavefront per atom.
//
// The paper names the ANI atom-centered symmetry functions as the operation
// its optimized kernels compute (Methods, "Optimization Through NNPOps"); the
// definition implemented is the published ANI one restated in nnp.h.  Forces
// are the negative gradient of the energy (Methods, "PyTorch Model Support").
//
// Per atom the wave first loads its neighbor records into LDS (displacement,
// distance, cutoff values, species).  Radial terms use lanes (g, m): four
// neighbors at a time, one radial shift m per lane; per-species sums stay in
// registers and are combined across the four neighbor slots by lane shuffles.
// Angular terms are enumerated per unordered species-pair block: the neighbor
// list is grouped by species, so the triples of block (p, q) are the products
// of two species segments (or the pairs inside one).  Lanes (t, z) take eight
// triples at a time, one angle shift z per lane, and keep the four radial
// shifts in registers; the block's 32 sums are combined across triple slots
// by shuffles and written once, so every output element is written by one
// store in a fixed summation order.  The angle term uses the identity
// cos(theta - theta_z) = kappa c cos(theta_z) + sqrt(1 - kappa^2 c^2) sin(theta_z)
// for theta = acos(kappa c); (1 + cos)/2 raised to zeta is exp2(zeta log2(.)).
//
// The adjoint recomputes the same terms, contracts them with g = dE/dG
// (read from the network backward pass), accumulates dE/d(displacement) per
// neighbor slot in LDS, then scatters: one atomic add per neighbor and
// component for the neighbors, and one wave-reduced add for the centre atom.
#include "kernels.h"

namespace nnp {

struct NbrLds {
  float4* d;    // dx, dy, dz, r
  float4* fc;   // fc_rad, fc_ang, dfc_rad, dfc_ang
  int* sp;
};

__device__ __forceinline__ float cutoff_val(float r, float inv_rc, float& dfc, float pi_2rc) {
  float s, c;
  sincospif(r * inv_rc, &s, &c);
  dfc = -pi_2rc * s;
  return 0.5f * c + 0.5f;
}

// Loads neighbor records of atom i into LDS; returns (nr, na).
__device__ __forceinline__ int2 load_neighbors(const AevConst& C, const BoxConst& B, int i,
                                               const float4* __restrict__ xyzs,
                                               const int* __restrict__ nbr,
                                               const int2* __restrict__ counts, int cap, int n,
                                               NbrLds L) {
  const int lane = lane_id();
  const int2 cn = counts[i];
  const int nr = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na = cn.y < 0 ? 0 : (cn.y > nr ? nr : cn.y);
  const float4 pi = xyzs[i];
  for (int e = lane; e < nr; e += kWave) {
    const int j = clampi(nbr[(size_t)i * cap + e], n);
    const float4 pj = xyzs[j];
    const float dx = disp(pi.x, pj.x, B.L[0], B.invL[0], B.periodic);
    const float dy = disp(pi.y, pj.y, B.L[1], B.invL[1], B.periodic);
    const float dz = disp(pi.z, pj.z, B.L[2], B.invL[2], B.periodic);
    const float r = sqrtf(dist2(dx, dy, dz));
    float dfr, dfa = 0.f;
    const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
    float fa = 0.f;
    if (e < na) fa = cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a);
    L.d[e] = make_float4(dx, dy, dz, r);
    L.fc[e] = make_float4(fr, fa, dfr, dfa);
    L.sp[e] = species_of(pj);
  }
  return make_int2(nr, na);
}

// Start of each species segment among the angular entries [0, na) (the list
// is grouped by species there).  Lane q < 9 returns the first index whose
// species is >= q.
__device__ __forceinline__ int segment_start(const int* sp, int na, int q) {
  int lo = 0, hi = na;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sp[mid] < q) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Triple t of block (p, q) -> entries (ej, ek) of the neighbor list.
__device__ __forceinline__ void decode_triple(int t, bool same, int sp0, int cp, int sq0, int cq,
                                              int& ej, int& ek) {
  if (!same) {
    const int a = t / cq;
    ej = sp0 + a;
    ek = sq0 + (t - a * cq);
    return;
  }
  // pairs a < b of one segment, row-major: start(a) = a*cp - a*(a+1)/2
  const float c2 = (float)(2 * cp - 1);
  int a = (int)((c2 - sqrtf(fmaxf(c2 * c2 - 8.f * (float)t, 0.f))) * 0.5f);
  a = a < 0 ? 0 : (a > cp - 2 ? cp - 2 : a);
  while (a > 0 && a * cp - a * (a + 1) / 2 > t) --a;
  while (a + 1 <= cp - 2 && (a + 1) * cp - (a + 1) * (a + 2) / 2 <= t) ++a;
  const int b = t - (a * cp - a * (a + 1) / 2) + a + 1;
  ej = sp0 + a;
  ek = sp0 + b;
}

__device__ __forceinline__ float sel8(const float (&v)[kMaxS], int q) {
  float r = v[0];
#pragma unroll
  for (int k = 1; k < kMaxS; ++k) r = (q == k) ? v[k] : r;
  return r;
}

__device__ __forceinline__ float sel4(float a0, float a1, float a2, float a3, int q) {
  return q == 0 ? a0 : (q == 1 ? a1 : (q == 2 ? a2 : a3));
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

template <typename OutT>
__global__ __launch_bounds__(256) void k_aev_fwd(const int* __restrict__ dims, AevConst C, BoxConst B,
                                                 const float4* __restrict__ xyzs,
                                                 const int* __restrict__ nbr,
                                                 const int2* __restrict__ counts, int cap,
                                                 const int* __restrict__ row_of,
                                                 OutT* __restrict__ out, int ld) {
  extern __shared__ float4 lds4[];
  const int n = dims[0];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  NbrLds L;
  L.d = lds4 + (size_t)w * cap * 2;
  L.fc = L.d + cap;
  L.sp = reinterpret_cast<int*>(lds4 + (size_t)4 * cap * 2) + w * cap;
  const int2 cnt = load_neighbors(C, B, i, xyzs, nbr, counts, cap, n, L);
  const int nr = cnt.x, na = cnt.y;
  wave_lds_sync();
  OutT* orow = out + (size_t)(row_of ? row_of[i] : i) * ld;
  const int S = C.S;

  // ---- radial
  {
    const int g = lane >> 4, m = lane & 15;
    const float Rm = C.shf_r[m];
    float acc[kMaxS];
#pragma unroll
    for (int q = 0; q < kMaxS; ++q) acc[q] = 0.f;
    for (int e = g; e < nr; e += 4) {
      const float r = L.d[e].w;
      const float fr = L.fc[e].x;
      const int s = L.sp[e];
      const float u = r - Rm;
      const float term = C.cR * fast_exp2(-C.eta_r_l2e * u * u) * fr;
#pragma unroll
      for (int q = 0; q < kMaxS; ++q) acc[q] += (s == q) ? term : 0.f;
    }
#pragma unroll
    for (int q = 0; q < kMaxS; ++q) {
      acc[q] += __shfl_xor(acc[q], 16, 64);
      acc[q] += __shfl_xor(acc[q], 32, 64);
    }
    const float v0 = sel8(acc, g), v1 = sel8(acc, g + 4);
    if (g < S) Store<OutT>::put(orow + g * kNR + m, v0);
    if (g + 4 < S) Store<OutT>::put(orow + (g + 4) * kNR + m, v1);
  }

  // ---- angular
  const int seg_mine = lane <= kMaxS ? segment_start(L.sp, na, lane) : na;
  const int tz = lane & 7, tg = lane >> 3;
  const float cz = C.cos_z[tz], sz = C.sin_z[tz];
  const float ra0 = C.shf_a[0], ra1 = C.shf_a[1], ra2 = C.shf_a[2], ra3 = C.shf_a[3];
  int blk = 0;
  for (int p = 0; p < S; ++p) {
    const int sp0 = __shfl(seg_mine, p, 64);
    const int cp = __shfl(seg_mine, p + 1, 64) - sp0;
    for (int q = p; q < S; ++q, ++blk) {
      const int sq0 = __shfl(seg_mine, q, 64);
      const int cq = __shfl(seg_mine, q + 1, 64) - sq0;
      const bool same = p == q;
      const int T = same ? cp * (cp - 1) / 2 : cp * cq;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      for (int t0 = 0; t0 < T; t0 += 8) {
        const int t = t0 + tg;
        if (t < T) {
          int ej, ek;
          decode_triple(t, same, sp0, cp, sq0, cq, ej, ek);
          const float4 vj = L.d[ej], vk = L.d[ek];
          const float fj = L.fc[ej].y, fk = L.fc[ek].y;
          const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) / (vj.w * vk.w);
          const float kc = C.kappa * cs;
          const float sn = sqrtf(fmaxf(1.f - kc * kc, 0.f));
          const float cd = kc * cz + sn * sz;
          const float base = 0.5f + 0.5f * cd;
          const float f1 = 2.f * fast_exp2(C.zeta * fast_log2(base));
          const float dbar = 0.5f * (vj.w + vk.w);
          const float wgt = f1 * fj * fk;
          float u;
          u = dbar - ra0; a0 += wgt * fast_exp2(-C.eta_a_l2e * u * u);
          u = dbar - ra1; a1 += wgt * fast_exp2(-C.eta_a_l2e * u * u);
          u = dbar - ra2; a2 += wgt * fast_exp2(-C.eta_a_l2e * u * u);
          u = dbar - ra3; a3 += wgt * fast_exp2(-C.eta_a_l2e * u * u);
        }
      }
#pragma unroll
      for (int o = 8; o <= 32; o <<= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
        a3 += __shfl_xor(a3, o, 64);
      }
      if (lane < 32) {
        const float v = sel4(a0, a1, a2, a3, lane >> 3);
        Store<OutT>::put(orow + S * kNR + blk * 32 + lane, v);
      }
    }
  }
  for (int c = C.F + lane; c < ld; c += kWave) Store<OutT>::put(orow + c, 0.f);
}

// Adjoint: g (float32 rows, stride ldg) -> scatter into out (float32 [n][3]).
// sign = +1 writes forces (-dE/dr); sign = -1 writes the gradient dE/dr.
__global__ __launch_bounds__(256) void k_aev_bwd(const int* __restrict__ dims, AevConst C, BoxConst B,
                                                 const float4* __restrict__ xyzs,
                                                 const int* __restrict__ nbr,
                                                 const int2* __restrict__ counts, int cap,
                                                 const int* __restrict__ row_of,
                                                 const float* __restrict__ g, int ldg,
                                                 float* __restrict__ out, float sign) {
  extern __shared__ float4 lds4[];
  const int n = dims[0];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  NbrLds L;
  L.d = lds4 + (size_t)w * cap * 3;
  L.fc = L.d + cap;
  float4* grad = L.fc + cap;
  L.sp = reinterpret_cast<int*>(lds4 + (size_t)4 * cap * 3) + w * cap;
  const int2 cnt = load_neighbors(C, B, i, xyzs, nbr, counts, cap, n, L);
  const int nr = cnt.x, na = cnt.y;
  const float* grow = g + (size_t)row_of[i] * ldg;
  const int S = C.S;

  // ---- radial: dE/dr_ij per neighbor, reduced over the 16 shift lanes
  {
    const int gq = lane >> 4, m = lane & 15;
    const float Rm = C.shf_r[m];
    wave_lds_sync();
    for (int e0 = 0; e0 < nr; e0 += 4) {
      const int e = e0 + gq;
      float contrib = 0.f;
      float4 v = make_float4(0.f, 0.f, 0.f, 1.f);
      if (e < nr) {
        v = L.d[e];
        const float4 f = L.fc[e];
        const int s = L.sp[e];
        const float u = v.w - Rm;
        const float ex = C.cR * fast_exp2(-C.eta_r_l2e * u * u);
        contrib = grow[s * kNR + m] * ex * (f.z - C.eta_r2 * u * f.x);
      }
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) contrib += __shfl_xor(contrib, o, 64);
      if (e < nr && m == 0) {
        const float sc = contrib / v.w;
        grad[e] = make_float4(v.x * sc, v.y * sc, v.z * sc, 0.f);
      }
    }
    wave_lds_sync();
  }

  // ---- angular
  const int seg_mine = lane <= kMaxS ? segment_start(L.sp, na, lane) : na;
  const int tz = lane & 7, tg = lane >> 3;
  const float cz = C.cos_z[tz], sz = C.sin_z[tz];
  const float ra0 = C.shf_a[0], ra1 = C.shf_a[1], ra2 = C.shf_a[2], ra3 = C.shf_a[3];
  int blk = 0;
  for (int p = 0; p < S; ++p) {
    const int sp0 = __shfl(seg_mine, p, 64);
    const int cp = __shfl(seg_mine, p + 1, 64) - sp0;
    for (int q = p; q < S; ++q, ++blk) {
      const int sq0 = __shfl(seg_mine, q, 64);
      const int cq = __shfl(seg_mine, q + 1, 64) - sq0;
      const bool same = p == q;
      const int T = same ? cp * (cp - 1) / 2 : cp * cq;
      if (T == 0) continue;
      const float* gb = grow + S * kNR + blk * 32 + tz;
      const float g0 = gb[0], g1 = gb[8], g2 = gb[16], g3 = gb[24];
      for (int t0 = 0; t0 < T; t0 += 8) {
        const int t = t0 + tg;
        float X0 = 0.f, X1 = 0.f, Xc = 0.f;
        int ej = 0, ek = 0;
        float4 vj = make_float4(0.f, 0.f, 0.f, 1.f), vk = vj;
        float fj = 0.f, fk = 0.f, dfj = 0.f, dfk = 0.f, cs = 0.f;
        if (t < T) {
          decode_triple(t, same, sp0, cp, sq0, cq, ej, ek);
          vj = L.d[ej];
          vk = L.d[ek];
          const float4 cj = L.fc[ej], ck = L.fc[ek];
          fj = cj.y; fk = ck.y; dfj = cj.w; dfk = ck.w;
          cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) / (vj.w * vk.w);
          const float kc = C.kappa * cs;
          const float sn = sqrtf(fmaxf(1.f - kc * kc, 1e-12f));
          const float cd = kc * cz + sn * sz;
          const float base = 0.5f + 0.5f * cd;
          const float pw = fast_exp2(C.zeta * fast_log2(base));
          const float f1 = 2.f * pw;
          // d f1 / d c = 2 zeta base^(zeta-1) * 0.5 * d cd / d c
          const float dcd = C.kappa * (cz - kc * sz / sn);
          const float df1 = C.zeta * pw / base * dcd;
          const float dbar = 0.5f * (vj.w + vk.w);
          float u, e2, A0 = 0.f, A1 = 0.f;
          u = dbar - ra0; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g0 * e2; A1 -= g0 * C.eta_a * u * e2;
          u = dbar - ra1; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g1 * e2; A1 -= g1 * C.eta_a * u * e2;
          u = dbar - ra2; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g2 * e2; A1 -= g2 * C.eta_a * u * e2;
          u = dbar - ra3; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g3 * e2; A1 -= g3 * C.eta_a * u * e2;
          X0 = f1 * A0;
          X1 = f1 * A1;
          Xc = df1 * A0;
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
          X0 += __shfl_xor(X0, o, 64);
          X1 += __shfl_xor(X1, o, 64);
          Xc += __shfl_xor(Xc, o, 64);
        }
        if (t < T && tz == 0) {
          const float fcc = fj * fk;
          const float dEdc = Xc * fcc;
          const float dEdj = X1 * fcc + X0 * dfj * fk;
          const float dEdk = X1 * fcc + X0 * fj * dfk;
          const float ijk = 1.f / (vj.w * vk.w);
          const float ij2 = 1.f / (vj.w * vj.w), ik2 = 1.f / (vk.w * vk.w);
          const float aj = dEdj / vj.w - dEdc * cs * ij2;
          const float ak = dEdk / vk.w - dEdc * cs * ik2;
          const float b = dEdc * ijk;
          atomicAdd(&grad[ej].x, aj * vj.x + b * vk.x);
          atomicAdd(&grad[ej].y, aj * vj.y + b * vk.y);
          atomicAdd(&grad[ej].z, aj * vj.z + b * vk.z);
          atomicAdd(&grad[ek].x, ak * vk.x + b * vj.x);
          atomicAdd(&grad[ek].y, ak * vk.y + b * vj.y);
          atomicAdd(&grad[ek].z, ak * vk.z + b * vj.z);
        }
      }
    }
  }
  wave_lds_sync();

  // ---- scatter: neighbors get -sign * dE/dv, the centre gets +sign * sum
  float sx = 0.f, sy = 0.f, sz2 = 0.f;
  for (int e = lane; e < nr; e += kWave) {
    const float4 gv = grad[e];
    const int j = clampi(nbr[(size_t)i * cap + e], n);
    unsafeAtomicAdd(out + 3 * j, -sign * gv.x);
    unsafeAtomicAdd(out + 3 * j + 1, -sign * gv.y);
    unsafeAtomicAdd(out + 3 * j + 2, -sign * gv.z);
    sx += gv.x;
    sy += gv.y;
    sz2 += gv.z;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz2 = wave_sum(sz2);
  if (lane == 0) {
    unsafeAtomicAdd(out + 3 * i, sign * sx);
    unsafeAtomicAdd(out + 3 * i + 1, sign * sy);
    unsafeAtomicAdd(out + 3 * i + 2, sign * sz2);
  }
}

// ----------------------------------------------------------------- launchers

template <typename OutT>
void launch_aev_fwd(const int* dims, int n_cap, const AevConst& C, const BoxConst& B,
                    const float4* xyzs, const int* nbr, const int2* counts, int cap,
                    const int* row_of, OutT* out, int ld, hipStream_t st) {
  if (n_cap <= 0) return;
  const size_t lds = (size_t)4 * cap * (2 * sizeof(float4) + sizeof(int));
  hipLaunchKernelGGL(k_aev_fwd<OutT>, dim3((n_cap + 3) / 4), dim3(256), lds, st, dims, C, B,
                     xyzs, nbr, counts, cap, row_of, out, ld);
}

template void launch_aev_fwd<float>(const int*, int, const AevConst&, const BoxConst&,
                                    const float4*, const int*, const int2*, int, const int*,
                                    float*, int, hipStream_t);
template void launch_aev_fwd<bf16_t>(const int*, int, const AevConst&, const BoxConst&,
                                     const float4*, const int*, const int2*, int, const int*,
                                     bf16_t*, int, hipStream_t);

void launch_aev_bwd(const int* dims, int n_cap, const AevConst& C, const BoxConst& B,
                    const float4* xyzs, const int* nbr, const int2* counts, int cap,
                    const int* row_of, const float* g, int ldg, float* out, float sign,
                    hipStream_t st) {
  if (n_cap <= 0) return;
  const size_t lds = (size_t)4 * cap * (3 * sizeof(float4) + sizeof(int));
  hipLaunchKernelGGL(k_aev_bwd, dim3((n_cap + 3) / 4), dim3(256), lds, st, dims, C, B, xyzs, nbr,
                     counts, cap, row_of, g, ldg, out, sign);
}

}  // namespace nnp

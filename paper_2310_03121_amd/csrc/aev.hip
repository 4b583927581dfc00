// Atomic environment vectors (forward) and their adjoint with the force
// scatter, one wavefront per atom.
//
// The paper names the ANI atom-centered symmetry functions as the operation
// its optimized kernels compute (Methods, "Optimization Through NNPOps"); the
// definition implemented is the published ANI one restated in nnp.h.  Forces
// are the negative gradient of the energy (Methods, "PyTorch Model Support").
//
// Per atom the wave first loads its neighbor records into LDS (displacement,
// distance, cutoff values, species).  Both sums of the forward pass are
// products with a one-hot matrix, which the FP32 MFMA computes exactly (its
// products are a term times 1 or 0): the radial row G[s][m] is
// onehot(species x neighbors) * terms(neighbors x 16 shifts), four neighbors
// per v_mfma_f32_16x16x4f32, and the angular rows G[block][a z] are
// onehot(blocks x pairs) * terms(pairs x 32), four neighbor pairs per pass.
// Each lane computes one term per product; there are no per-block loops or
// cross-lane reductions, and the accumulator layout is the feature layout,
// so the results are stored straight from registers.  The angle term uses
// the identity
// cos(theta - theta_z) = kappa c cos(theta_z) + sqrt(1 - kappa^2 c^2) sin(theta_z)
// for theta = acos(kappa c); (1 + cos)/2 raised to zeta is exp2(zeta log2(.)).
//
// The adjoint recomputes the same terms, contracts them with g = dE/dG
// (read from the network backward pass, only the blocks the atom touches),
// accumulates dE/d(displacement) per neighbor slot in LDS, then scatters: one
// atomic add per neighbor and component for the neighbors, and one
// wave-reduced add for the centre atom.
#include "kernels.h"
#include "energy_sum.h"

namespace nnp {

// sin(pi t) and cos(pi t) for t in [0, 1] from Taylor polynomials of sin and
// cos on u = pi (t - 1/2) in [-pi/2, pi/2] (cos(pi t) = -sin u,
// sin(pi t) = cos u); the truncation error is below 1e-8, under FP32 rounding.
__device__ __forceinline__ void sincos_pi01(float t, float& s, float& c) {
  const float u = 3.14159265358979f * (t - 0.5f);
  const float u2 = u * u;
  // sin u = u (1 - u^2/3! + u^4/5! - ... - u^12/13!)
  float ps = -1.6059043836821614e-10f;               // -1/13!
  ps = ps * u2 + 2.5052108385441720e-8f;              //  1/11!
  ps = ps * u2 - 2.7557319223985893e-6f;              // -1/9!
  ps = ps * u2 + 1.9841269841269841e-4f;              //  1/7!
  ps = ps * u2 - 8.3333333333333333e-3f;              // -1/5!
  ps = ps * u2 + 1.6666666666666667e-1f;              //  1/3!
  const float sinu = u - u * u2 * ps;
  // cos u = 1 - u^2/2! + u^4/4! - ... + u^12/12!
  float pc = 2.0876756987868099e-9f;                 //  1/12!
  pc = pc * u2 - 2.7557319223985891e-7f;              // -1/10!
  pc = pc * u2 + 2.4801587301587302e-5f;              //  1/8!
  pc = pc * u2 - 1.3888888888888889e-3f;              // -1/6!
  pc = pc * u2 + 4.1666666666666667e-2f;              //  1/4!
  pc = pc * u2 - 0.5f;                                // -1/2!
  const float cosu = 1.f + u2 * pc;
  c = -sinu;
  s = cosu;
}

// fc(r; R) = cos(pi r / R)/2 + 1/2 and its derivative -(pi/2R) sin(pi r/R).
__device__ __forceinline__ float cutoff_val(float r, float inv_rc, float& dfc, float pi_2rc) {
  float s, c;
  sincos_pi01(fminf(r * inv_rc, 1.f), s, c);
  dfc = -pi_2rc * s;
  return 0.5f * c + 0.5f;
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Records read before the neighbor count is known: enough for a molecule's
// atoms (up to 16 neighbors) without fetching the whole 64-entry window.
constexpr int kSpecRec = 16;

// v_sqrt_f32 (about 1 ulp): neighbor distances and the angle sine are
// normal numbers, so the IEEE-exact expansion (denormal scaling and two
// correction steps) buys nothing here
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Unordered pair t of the list prefix [0, na) -> entries a < b, row-major:
// row r starts at pair r (2 na - r - 1) / 2.  The row is the floor of the
// smaller root of that quadratic; the float square root (exact operands for
// na <= 2048) can put it one row off either way near a row start, which one
// compare-and-select step in each direction corrects.  Branch-free, so the
// lanes of a pass never diverge.
__device__ __forceinline__ void decode_pair(int t, int na, int& a, int& b) {
  const float c2 = (float)(2 * na - 1);
  int r = (int)((c2 - fast_sqrt(fmaxf(c2 * c2 - 8.f * (float)t, 0.f))) * 0.5f);
  r = r < 0 ? 0 : (r > na - 2 ? na - 2 : r);
  r = (r * (2 * na - r - 1)) >> 1 > t ? r - 1 : r;
  const bool up = (r + 1 <= na - 2) & ((((r + 1) * (2 * na - r - 2)) >> 1) <= t);
  r = up ? r + 1 : r;
  a = r;
  b = t - ((r * (2 * na - r - 1)) >> 1) + r + 1;
}

__device__ __forceinline__ int pair_block(int p, int q, int S) {
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  return lo * S - lo * (lo - 1) / 2 + (hi - lo);
}

// Angular pairs are decoded in chunks of 64, one pair per lane, into a
// per-wave LDS table that the passes then read.
constexpr int kPairChunk = 64;

// LDS per wave (forward): per neighbor float4 (dx, dy, dz, r), float2
// (fc_rad, fc_ang), int species; a 64-entry table of angular pairs (float4
// geometry and int block each).  The feature row is accumulated in registers
// and stored block by block, so no LDS row is needed.
constexpr int kFwdBytesPerNbr = 16 + 8 + 4;
constexpr int kFwdPairBytes = 16 + 4;

// The angular pairs [c0, c0 + 64) of the list, one per lane: what a pair's
// 32 terms share, computed once instead of in each of the 16 lanes of its
// pass: (kappa cos theta, sqrt(1 - kappa^2 cos^2), mean distance,
// fc_j fc_k) and the pair's block.
__device__ __forceinline__ void pair_chunk_geometry(int c0, int T, int na, const AevConst& C,
                                                    const float4* nd, const float2* nf,
                                                    const int* nsp, float4* pgeo, int* pblk,
                                                    int lane) {
  const int t = c0 + lane;
  if (t < T) {
    int a, b;
    decode_pair(t, na, a, b);
    const float4 vj = nd[a], vk = nd[b];
    const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) * fast_rcp(vj.w * vk.w);
    const float kc = C.kappa * cs;
    pgeo[lane] = make_float4(kc, fast_sqrt(fmaxf(1.f - kc * kc, 0.f)), 0.5f * (vj.w + vk.w),
                             nf[a].y * nf[b].y);
    pblk[lane] = pair_block(nsp[a], nsp[b], C.S);
  }
}

typedef float aev_f32x4 __attribute__((ext_vector_type(4)));

// acc += A * B for one 16 x 16 x 4 FP32 MFMA: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds C[4 * (l / 16) + r][l % 16], r = 0..3.  The
// forward pass passes the terms as A and the one-hot as B, so C is the
// transposed feature block: lane l holds features 4 (l / 16) .. +3 of
// species (or block) l % 16, stored as one vector.
__device__ __forceinline__ aev_f32x4 mfma4(float a, float b, aev_f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// NT: 16-block tiles of the angular one-hot (ceil(S (S + 1) / 2 / 16): one
// for up to five elements, two for six or seven, three for eight).
template <typename OutT, int NT>
__global__ __launch_bounds__(256) void k_aev_fwd(const int* __restrict__ dims, AevConst C,
                                                 const float4* __restrict__ rec,
                                                 const int2* __restrict__ counts, int cap,
                                                 const int* __restrict__ row_of,
                                                 OutT* __restrict__ out, int ld) {
  extern __shared__ float4 lds4[];
  const int n = dims[0];
  const int w = threadIdx.x >> 6;
  const int lane = lane_id();
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  float4* nd = lds4 + (size_t)w * cap;
  float2* nf = reinterpret_cast<float2*>(lds4 + (size_t)4 * cap) + (size_t)w * cap;
  int* nsp = reinterpret_cast<int*>(reinterpret_cast<float2*>(lds4 + (size_t)4 * cap) +
                                    (size_t)4 * cap) + w * cap;
  float4* pgeo = reinterpret_cast<float4*>(
                     reinterpret_cast<int*>(reinterpret_cast<float2*>(lds4 + (size_t)4 * cap) +
                                            (size_t)4 * cap) + 4 * cap) + w * kPairChunk;
  int* pblk = reinterpret_cast<int*>(pgeo + (4 - w) * kPairChunk) + w * kPairChunk;

  // the first 64 records are fetched together with the counts
  const float4* nrec = rec + (size_t)i * cap;
  const float4 q0 = lane < kSpecRec && lane < cap ? nrec[lane] : make_float4(0.f, 0.f, 0.f, 0.f);
  const int2 cn = counts[i];
  const int nr = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na = cn.y < 0 ? 0 : (cn.y > nr ? nr : cn.y);
  auto setup = [&](int e, const float4 q) __attribute__((always_inline)) {
    const float r = fast_sqrt(dist2(q.x, q.y, q.z));
    float dfr, dfa;
    const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
    const float fa = e < na ? cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a) : 0.f;
    nd[e] = make_float4(q.x, q.y, q.z, r);
    nf[e] = make_float2(fr, fa);
    nsp[e] = species_of(q);
  };
  if (nr <= kSpecRec) {  // wave-uniform
    if (lane < nr) setup(lane, q0);
  } else {
    for (int e = lane; e < nr; e += kWave) setup(e, nrec[e]);
  }
  wave_lds_sync();
  const int S = C.S;
  OutT* orow = out + (size_t)(row_of ? row_of[i] : i) * ld;
  const int l16 = lane & 15, kq = lane >> 4;

  // ---- radial: G[s][m] = sum over neighbors e of [species(e) == s] * term(e, m)
  // as MFMA products of a one-hot (species x 4 neighbors) with the terms
  // (4 neighbors x 16 shifts); lane (kq, l16) computes neighbor kq, shift l16.
  {
    const float Rm = C.lane_tab[l16];
    aev_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int e0 = 0; e0 < nr; e0 += 4) {
      const int e = e0 + kq;
      float term = 0.f, hot = 0.f;
      if (e < nr) {
        const float u = nd[e].w - Rm;
        term = C.cR * fast_exp2(-C.eta_r_l2e * u * u) * nf[e].x;
        hot = nsp[e] == l16 ? 1.f : 0.f;
      }
      acc = mfma4(term, hot, acc);
    }
    if (l16 < S)
      Store<OutT>::put4(orow + l16 * kNR + 4 * kq, make_float4(acc[0], acc[1], acc[2], acc[3]));
  }

  // ---- angular: G[blk][a z] = sum over unordered pairs of angular neighbors
  // of [block(pair) == blk] * term(pair, a, z), four pairs per pass.  Lane
  // (kq, l16) takes pair kq and column l16 of each of the two 16-column
  // halves: angle shift z = l16 % 8 and radial shifts a = l16 / 8 and
  // l16 / 8 + 2.  Tile u of the one-hot covers blocks 16 u .. 16 u + 15.
  {
    const int T = na * (na - 1) / 2;
    const int nblk = S * (S + 1) / 2;
    const int z = l16 & 7, ah = l16 >> 3;
    const float cz = C.lane_tab[kNR + z], sz = C.lane_tab[kNR + kNZ + z];
    const float ra_lo = ah ? C.shf_a[1] : C.shf_a[0];
    const float ra_hi = ah ? C.shf_a[3] : C.shf_a[2];
    aev_f32x4 c0[NT], c1[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      c0[u] = aev_f32x4{0.f, 0.f, 0.f, 0.f};
      c1[u] = c0[u];
    }
    for (int p0 = 0; p0 < T; p0 += kPairChunk) {
    pair_chunk_geometry(p0, T, na, C, nd, nf, nsp, pgeo, pblk, lane);
    wave_lds_sync();
    const int tn = T - p0 < kPairChunk ? T - p0 : kPairChunk;
    for (int t0 = 0; t0 < tn; t0 += 4) {
      const int t = t0 + kq;
      float b0 = 0.f, b1 = 0.f;
      int blk = -1;
      if (t < tn) {
        const float4 q = pgeo[t];  // kappa cos, sine, mean distance, fc_j fc_k
        blk = pblk[t];
        const float base_ = 0.5f + 0.5f * (q.x * cz + q.y * sz);
        const float wgt = 2.f * fast_exp2(C.zeta * fast_log2(base_)) * q.w;
        const float u0 = q.z - ra_lo, u1 = q.z - ra_hi;
        b0 = wgt * fast_exp2(-C.eta_a_l2e * u0 * u0);
        b1 = wgt * fast_exp2(-C.eta_a_l2e * u1 * u1);
      }
      // every tile's product runs on every pass: a tile without the pass's
      // blocks adds zeros, which costs less than a branch that keeps the
      // accumulators apart
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const float hot = blk == l16 + 16 * u ? 1.f : 0.f;
        c0[u] = mfma4(b0, hot, c0[u]);
        c1[u] = mfma4(b1, hot, c1[u]);
      }
    }
    wave_lds_sync();  // the next chunk overwrites the table
    }
    // column c of c0[u] is feature c of block 16 u + l16 (a = c / 8 for the
    // low radial shifts, z = c % 8); c1[u] holds features 16 + c
    OutT* ang = orow + S * kNR + l16 * 32 + 4 * kq;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (l16 + 16 * u < nblk) {
        Store<OutT>::put4(ang + 512 * u, make_float4(c0[u][0], c0[u][1], c0[u][2], c0[u][3]));
        Store<OutT>::put4(ang + 512 * u + 16,
                          make_float4(c1[u][0], c1[u][1], c1[u][2], c1[u][3]));
      }
    }
  }
  for (int c = C.F + lane; c < ld; c += kWave) Store<OutT>::put(orow + c, 0.f);
}

// Atoms per workgroup of the molecule adjoint.
constexpr int kMolBlock = 64;

// LDS per wave (adjoint): per neighbor float4 (dx, dy, dz, r), float4
// (fc_rad, fc_ang, dfc_rad, dfc_ang), float4 accumulated dE/d(displacement),
// int species.  The dE/dG row is read from global memory where a term needs
// it (an atom touches only the blocks of the species around it).  Pairs are
// decoded per lane here: with eight lanes per pair the chunked table of the
// forward pass measured no gain.
constexpr int kBwdBytesPerNbr = 16 + 16 + 16 + 4;

// The adjoint of one atom i, by one wave: dE/d(displacement) of every
// neighbor entry into the wave's LDS region, then put(j, x, y, z) adds
// -sign * dE/dv to neighbor j and (lane 0) +sign * sum to the centre i.
// nd, nf, grad: cap float4 each; nsp: cap ints.
template <typename GT, typename Put>
__device__ __forceinline__ void adjoint_atom(int i, int n, const AevConst& C,
                                             const float4* __restrict__ rec,
                                             const int* __restrict__ nbr,
                                             const int2* __restrict__ counts, int cap,
                                             const int* __restrict__ row_of,
                                             const GT* __restrict__ g, int ldg, float sign,
                                             float4* nd, float4* nf, float4* grad, int* nsp,
                                             Put&& put) {
  const int lane = lane_id();
  // records, counts, the dE/dG row and the neighbor indices of the scatter
  // are all first-level loads
  const int* nrow = nbr + (size_t)i * cap;
  const float4* nrec = rec + (size_t)i * cap;
  const float4 q0 = lane < kSpecRec && lane < cap ? nrec[lane] : make_float4(0.f, 0.f, 0.f, 0.f);
  const int j0 = lane < kSpecRec && lane < cap ? nrow[lane] : 0;
  const int2 cn = counts[i];
  const GT* grow = g + (size_t)row_of[i] * ldg;
  const int nr = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na = cn.y < 0 ? 0 : (cn.y > nr ? nr : cn.y);
  auto setup = [&](int e, const float4 q) __attribute__((always_inline)) {
    const float r = fast_sqrt(dist2(q.x, q.y, q.z));
    float dfr, dfa = 0.f;
    const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
    const float fa = e < na ? cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a) : 0.f;
    nd[e] = make_float4(q.x, q.y, q.z, r);
    nf[e] = make_float4(fr, fa, dfr, dfa);
    nsp[e] = species_of(q);
  };
  if (nr <= kSpecRec) {  // wave-uniform
    if (lane < nr) setup(lane, q0);
  } else {
    for (int e = lane; e < nr; e += kWave) setup(e, nrec[e]);
  }
  wave_lds_sync();
  const int S = C.S;

  // ---- radial: dE/dr_ij per neighbor, reduced over the 16 shift lanes
  {
    const int gq = lane >> 4, m = lane & 15;
    const float Rm = C.lane_tab[m];
    for (int e0 = 0; e0 < nr; e0 += 4) {
      const int e = e0 + gq;
      float contrib = 0.f;
      float4 v = make_float4(0.f, 0.f, 0.f, 1.f);
      if (e < nr) {
        v = nd[e];
        const float4 f = nf[e];
        const float u = v.w - Rm;
        const float ex = C.cR * fast_exp2(-C.eta_r_l2e * u * u);
        contrib = Store<GT>::get(grow + nsp[e] * kNR + m) * ex * (f.z - C.eta_r2 * u * f.x);
      }
      contrib = group16_sum(contrib);
      if (e < nr && m == 0) {
        const float sc = contrib * fast_rcp(v.w);
        grad[e] = make_float4(v.x * sc, v.y * sc, v.z * sc, 0.f);
      }
    }
  }
  wave_lds_sync();

  // ---- angular: lanes (t, z), eight unordered pairs per pass
  {
    const int tz = lane & 7, tg = lane >> 3;
    const float cz = C.lane_tab[kNR + tz], sz = C.lane_tab[kNR + kNZ + tz];
    const float ra0 = C.shf_a[0], ra1 = C.shf_a[1], ra2 = C.shf_a[2], ra3 = C.shf_a[3];
    const int T = na * (na - 1) / 2;
    const GT* gang = grow + S * kNR + tz;
    for (int t0 = 0; t0 < T; t0 += 8) {
      // lanes past the last pair recompute it and contribute zero: every lane
      // runs the same straight-line code, with no branch around the terms
      const int t = t0 + tg;
      const bool valid = t < T;
      int ej, ek;
      decode_pair(valid ? t : T - 1, na, ej, ek);
      const float4 vj = nd[ej], vk = nd[ek];
      const float4 cj = nf[ej], ck = nf[ek];
      const float fj = cj.y, fk = ck.y, dfj = cj.w, dfk = ck.w;
      const GT* gb = gang + pair_block(nsp[ej], nsp[ek], S) * 32;
      const float g0 = Store<GT>::get(gb), g1 = Store<GT>::get(gb + 8),
                  g2 = Store<GT>::get(gb + 16), g3 = Store<GT>::get(gb + 24);
      const float rj = fast_rcp(vj.w), rk = fast_rcp(vk.w);
      const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) * (rj * rk);
      const float kc = C.kappa * cs;
      const float sn = fast_sqrt(fmaxf(1.f - kc * kc, 1e-12f));
      const float base_ = 0.5f + 0.5f * (kc * cz + sn * sz);
      const float pw = fast_exp2(C.zeta * fast_log2(base_));
      const float f1 = 2.f * pw;
      // d f1 / d c = zeta base^(zeta-1) d(kappa c cos_z + sqrt(1-kappa^2 c^2) sin_z)/dc
      const float df1 = C.zeta * pw * fast_rcp(base_) * (C.kappa * (cz - kc * sz * fast_rcp(sn)));
      const float dbar = 0.5f * (vj.w + vk.w);
      float u, e2, A0 = 0.f, A1 = 0.f;
      u = dbar - ra0; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g0 * e2; A1 -= g0 * u * e2;
      u = dbar - ra1; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g1 * e2; A1 -= g1 * u * e2;
      u = dbar - ra2; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g2 * e2; A1 -= g2 * u * e2;
      u = dbar - ra3; e2 = fast_exp2(-C.eta_a_l2e * u * u); A0 += g3 * e2; A1 -= g3 * u * e2;
      float X0 = valid ? f1 * A0 : 0.f;
      float X1 = valid ? f1 * A1 * C.eta_a : 0.f;
      float Xc = valid ? df1 * A0 : 0.f;
      X0 = group8_sum(X0);
      X1 = group8_sum(X1);
      Xc = group8_sum(Xc);
      if (valid && tz == 0) {
        const float fcc = fj * fk;
        const float dEdc = Xc * fcc;
        const float dEdj = X1 * fcc + X0 * dfj * fk;
        const float dEdk = X1 * fcc + X0 * fj * dfk;
        const float aj = (dEdj - dEdc * cs * rj) * rj;
        const float ak = (dEdk - dEdc * cs * rk) * rk;
        const float bb = dEdc * rj * rk;
        atomicAdd(&grad[ej].x, aj * vj.x + bb * vk.x);
        atomicAdd(&grad[ej].y, aj * vj.y + bb * vk.y);
        atomicAdd(&grad[ej].z, aj * vj.z + bb * vk.z);
        atomicAdd(&grad[ek].x, ak * vk.x + bb * vj.x);
        atomicAdd(&grad[ek].y, ak * vk.y + bb * vj.y);
        atomicAdd(&grad[ek].z, ak * vk.z + bb * vj.z);
      }
    }
  }
  wave_lds_sync();

  // ---- scatter: neighbors get -sign * dE/dv, the centre gets +sign * sum
  float sx = 0.f, sy = 0.f, sz2 = 0.f;
  for (int e = lane; e < nr; e += kWave) {
    const float4 gv = grad[e];
    put(clampi(e < kSpecRec ? j0 : nrow[e], n), -sign * gv.x, -sign * gv.y, -sign * gv.z);
    sx += gv.x;
    sy += gv.y;
    sz2 += gv.z;
  }
  sx = wave_sum_rows(sx);
  sy = wave_sum_rows(sy);
  sz2 = wave_sum_rows(sz2);
  if (lane == 0) put(i, sign * sx, sign * sy, sign * sz2);
}

// Adjoint: g (rows of type GT, stride ldg) -> scatter into out (float32 [n][3]).
// sign = +1 writes forces (-dE/dr); sign = -1 writes the gradient dE/dr.
// With gidx, atom i's force goes to row gidx[i] of out ([n_total][3]; rows
// outside [0, n_total) are skipped; staging reports them).  Blocks from
// nb_adj on sum the molecular energies (one block per molecule), which need
// only the atomic energies of the forward pass: they fill the tail of the
// scatter instead of a launch of their own.
template <typename GT>
__global__ __launch_bounds__(256) void k_aev_bwd(const int* __restrict__ dims, AevConst C,
                                                 const float4* __restrict__ rec,
                                                 const int* __restrict__ nbr,
                                                 const int2* __restrict__ counts, int cap,
                                                 const int* __restrict__ row_of,
                                                 const GT* __restrict__ g, int ldg,
                                                 float* __restrict__ out, float sign,
                                                 const int* __restrict__ gidx, int n_total,
                                                 int nb_adj, EnergyArgs EA) {
  extern __shared__ float4 lds4[];
  if ((int)blockIdx.x >= nb_adj) {  // block-uniform: the molecular energy sums
    energy_block((int)blockIdx.x - nb_adj, dims, EA);
    return;
  }
  const int n = dims[0];
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  float4* nd = lds4 + (size_t)w * cap * 3;
  int* nsp = reinterpret_cast<int*>(lds4 + (size_t)4 * cap * 3) + w * cap;
  adjoint_atom<GT>(i, n, C, rec, nbr, counts, cap, row_of, g, ldg, sign, nd, nd + cap,
                   nd + 2 * cap, nsp, [&](int j, float x, float y, float z) {
                     if (gidx) {
                       j = gidx[j];
                       if (j < 0 || j >= n_total) return;
                     }
                     unsafeAtomicAdd(out + 3 * j, x);
                     unsafeAtomicAdd(out + 3 * j + 1, y);
                     unsafeAtomicAdd(out + 3 * j + 2, z);
                   });
}

// Molecules (no box, no index map): a workgroup owns the kMolBlock atoms
// [b * kMolBlock, (b + 1) * kMolBlock), its waves taking them in turn, and
// adds every force into an LDS window over the atoms [b - 1, b + 2) *
// kMolBlock, which holds all neighbors of its atoms for molecules of up to
// kMolBlock + 1 atoms (neighbors outside it, in larger molecules, are added
// to global memory directly).  At the end each touched window atom is written
// once: with a plain store if its whole molecule lies inside the workgroup's
// atoms (nothing else adds to it; staging zeroed the output), else with one
// atomic add per component.  This replaces the contended per-entry global
// atomics of the per-atom kernel (about nine adds per atom on the same lines).
template <typename GT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_aev_bwd_mol(const int* __restrict__ dims, AevConst C,
                                                      const float4* __restrict__ rec,
                                                      const int* __restrict__ nbr,
                                                      const int2* __restrict__ counts, int cap,
                                                      const int* __restrict__ row_of,
                                                      const GT* __restrict__ g, int ldg,
                                                      float* __restrict__ out, float sign,
                                                      const int2* __restrict__ mrange,
                                                      int nb_adj, EnergyArgs EA) {
  extern __shared__ float4 lds4[];
  if ((int)blockIdx.x >= nb_adj) {  // block-uniform: the molecular energy sums
    energy_block((int)blockIdx.x - nb_adj, dims, EA);
    return;
  }
  constexpr int kWin = 3 * kMolBlock;
  const int n = dims[0];
  const int nw = (int)blockDim.x >> 6, w = (int)threadIdx.x >> 6;
  const int base = (int)blockIdx.x * kMolBlock, w0 = base - kMolBlock;
  float4* nd = lds4 + (size_t)w * cap * 3;
  int* nsp = reinterpret_cast<int*>(lds4 + (size_t)nw * cap * 3) + w * cap;
  float* win = reinterpret_cast<float*>(reinterpret_cast<int*>(lds4 + (size_t)nw * cap * 3) +
                                        (size_t)nw * cap);
  for (int t = threadIdx.x; t < 3 * kWin; t += blockDim.x) win[t] = 0.f;
  __syncthreads();
  for (int a = w; a < kMolBlock; a += nw) {
    const int i = base + a;
    if (i >= n) break;  // wave-uniform
    adjoint_atom<GT>(i, n, C, rec, nbr, counts, cap, row_of, g, ldg, sign, nd, nd + cap,
                     nd + 2 * cap, nsp, [&](int j, float x, float y, float z) {
                       const int t = j - w0;
                       if (t >= 0 && t < kWin) {
                         atomicAdd(win + 3 * t, x);
                         atomicAdd(win + 3 * t + 1, y);
                         atomicAdd(win + 3 * t + 2, z);
                       } else {
                         unsafeAtomicAdd(out + 3 * j, x);
                         unsafeAtomicAdd(out + 3 * j + 1, y);
                         unsafeAtomicAdd(out + 3 * j + 2, z);
                       }
                     });
    wave_lds_sync();  // the next atom reuses this wave's region
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kWin; t += blockDim.x) {
    const int j = w0 + t;
    if (j < 0 || j >= n) continue;
    const float x = win[3 * t], y = win[3 * t + 1], z = win[3 * t + 2];
    if (x == 0.f && y == 0.f && z == 0.f) continue;
    const int2 mr = mrange[j];
    if (mr.x >= base && mr.y <= base + kMolBlock) {
      out[3 * j] = x;
      out[3 * j + 1] = y;
      out[3 * j + 2] = z;
    } else {
      unsafeAtomicAdd(out + 3 * j, x);
      unsafeAtomicAdd(out + 3 * j + 1, y);
      unsafeAtomicAdd(out + 3 * j + 2, z);
    }
  }
}

// ----------------------------------------------------------------- launchers

template <typename OutT>
void launch_aev_fwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int2* counts, int cap, const int* row_of, OutT* out, int ld,
                    hipStream_t st) {
  if (n_cap <= 0) return;
  const size_t lds = (size_t)4 * cap * kFwdBytesPerNbr + (size_t)4 * kPairChunk * kFwdPairBytes;
  static const bool attr = (ensure_lds(k_aev_fwd<OutT, 1>), ensure_lds(k_aev_fwd<OutT, 2>),
                            ensure_lds(k_aev_fwd<OutT, 3>), true);
  (void)attr;
  const int nblk = C.S * (C.S + 1) / 2;
  auto kern = nblk <= 16 ? k_aev_fwd<OutT, 1> : (nblk <= 32 ? k_aev_fwd<OutT, 2>
                                                             : k_aev_fwd<OutT, 3>);
  hipLaunchKernelGGL(kern, dim3((n_cap + 3) / 4), dim3(256), lds, st, dims, C, rec, counts, cap,
                     row_of, out, ld);
}
template void launch_aev_fwd<float>(const int*, int, const AevConst&, const float4*, const int2*,
                                    int, const int*, float*, int, hipStream_t);
template void launch_aev_fwd<bf16_t>(const int*, int, const AevConst&, const float4*,
                                     const int2*, int, const int*, bf16_t*, int, hipStream_t);

template <typename GT>
void launch_aev_bwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int* nbr, const int2* counts, int cap, const int* row_of, const GT* g,
                    int ldg, float* out, float sign, const int* gidx, int n_total,
                    const int2* mrange, const EnergyArgs* energy, int nmol_cap,
                    hipStream_t st) {
  const int nb_e = energy && energy->E && nmol_cap > 0 ? nmol_cap : 0;
  const EnergyArgs ea = nb_e ? *energy : EnergyArgs{};
  if (mrange && !gidx) {
    // waves per workgroup: 16 while two workgroups fit a CU's LDS, else fewer
    const int nw = cap <= 64 ? 16 : (cap <= 128 ? 8 : 4);
    const int nb_adj = n_cap > 0 ? (n_cap + kMolBlock - 1) / kMolBlock : 0;
    if (nb_adj + nb_e == 0) return;
    const size_t lds = (size_t)nw * cap * kBwdBytesPerNbr + (size_t)3 * kMolBlock * 3 * 4;
    static const bool attr = (ensure_lds(k_aev_bwd_mol<GT>), true);
    (void)attr;
    hipLaunchKernelGGL(k_aev_bwd_mol<GT>, dim3(nb_adj + nb_e), dim3(64 * nw), lds, st, dims, C,
                       rec, nbr, counts, cap, row_of, g, ldg, out, sign, mrange, nb_adj, ea);
    return;
  }
  const int nb_adj = n_cap > 0 ? (n_cap + 3) / 4 : 0;
  if (nb_adj + nb_e == 0) return;
  const size_t lds = (size_t)4 * cap * kBwdBytesPerNbr;
  static const bool attr = (ensure_lds(k_aev_bwd<GT>), true);
  (void)attr;
  hipLaunchKernelGGL(k_aev_bwd<GT>, dim3(nb_adj + nb_e), dim3(256), lds, st, dims, C, rec, nbr,
                     counts, cap, row_of, g, ldg, out, sign, gidx, n_total, nb_adj, ea);
}
template void launch_aev_bwd<float>(const int*, int, const AevConst&, const float4*, const int*,
                                    const int2*, int, const int*, const float*, int, float*, float,
                                    const int*, int, const int2*, const EnergyArgs*, int,
                                    hipStream_t);
template void launch_aev_bwd<bf16_t>(const int*, int, const AevConst&, const float4*, const int*,
                                     const int2*, int, const int*, const bf16_t*, int, float*,
                                     float, const int*, int, const int2*, const EnergyArgs*, int,
                                     hipStream_t);

}  // namespace nnp

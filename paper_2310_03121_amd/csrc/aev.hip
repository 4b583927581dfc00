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
// (fc_rad, fc_ang), int species; a 64-entry table of angular pairs (eight
// angle-shift weights, four distance Gaussians and the block of each).  The
// feature row is accumulated in registers and stored block by block, so no
// LDS row is needed.
constexpr int kFwdBytesPerNbr = 16 + 8 + 4;
constexpr int kFwdPairBytes = 32 + 16 + 4;

typedef float aev_f32x4 __attribute__((ext_vector_type(4)));

// acc += A * B for one 16 x 16 x 4 FP32 MFMA: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and holds C[4 * (l / 16) + r][l % 16], r = 0..3.  The
// forward pass passes the terms as A and the one-hot as B, so C is the
// transposed feature block: lane l holds features 4 (l / 16) .. +3 of
// species (or block) l % 16, stored as one vector.
__device__ __forceinline__ aev_f32x4 mfma4(float a, float b, aev_f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}

// The angular pair t of atom-local list prefix [0, na), one per lane: the
// factors of its 32 terms, computed once instead of in each of the 16 lanes
// of its pass, written to table slot `slot`: the angle-shift weights
// w[z] = 2 ((1 + cos(theta - theta_z)) / 2)^zeta fc_j fc_k and the distance
// Gaussians g[a] = exp(-eta_A ((r_j + r_k) / 2 - R_a)^2); term (a, z) = w[z] g[a].
__device__ __forceinline__ void pair_geometry(int t, int na, const AevConst& C, const float4* nd,
                                              const float2* nf, const int* nsp, float* pw,
                                              float* pg, int* pblk, int slot) {
  int a, b;
  decode_pair(t, na, a, b);
  const float4 vj = nd[a], vk = nd[b];
  const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) * fast_rcp(vj.w * vk.w);
  const float kc = C.kappa * cs;
  const float sn = fast_sqrt(fmaxf(1.f - kc * kc, 0.f));
  const float dbar = 0.5f * (vj.w + vk.w);
  const float fcc = nf[a].y * nf[b].y;
  float w[kNZ];
#pragma unroll
  for (int z = 0; z < kNZ; ++z) {
    const float base_ = 0.5f + 0.5f * (kc * C.lane_tab[kNR + z] + sn * C.lane_tab[kNR + kNZ + z]);
    w[z] = 2.f * fast_exp2(C.zeta * fast_log2(base_)) * fcc;
  }
  float g[kNA];
#pragma unroll
  for (int q = 0; q < kNA; ++q) {
    const float u = dbar - C.shf_a[q];
    g[q] = fast_exp2(-C.eta_a_l2e * u * u);
  }
  reinterpret_cast<float4*>(pw)[2 * slot] = make_float4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<float4*>(pw)[2 * slot + 1] = make_float4(w[4], w[5], w[6], w[7]);
  reinterpret_cast<float4*>(pg)[slot] = make_float4(g[0], g[1], g[2], g[3]);
  pblk[slot] = pair_block(nsp[a], nsp[b], C.S);
}

// Four atoms per wave.  When each of a wave's four atoms has at most 16
// neighbors ("quad" waves), the per-neighbor setup (distances, cutoffs,
// species; in the adjoint also the force scatter and the centre-atom sum)
// runs for all four at once, one 16-lane group per atom, and the pairs of
// angular neighbors of all four share one table; the radial and angular
// passes, which fill the wave with (neighbor, shift) and (pair, shift) lanes,
// run atom by atom.  Other waves take their atoms one at a time with all 64
// lanes.  Either way a wave's LDS region holds max(64, capacity) neighbor
// entries: four 16-entry slots, or one atom's list.
//
// Quads pay off only where lists are short; where they are long, a wave per
// atom keeps four times as many waves in flight to hide the latency of the
// per-atom passes.  The launchers take the neighbor capacity as the hint:
// Q = 4 atoms per wave up to a capacity of 64 (molecules), else Q = 1
// (liquid-density boxes need more than 64).
constexpr int kQuadNbr = 16;   // longest list of a quad wave (lanes per atom)

__host__ __device__ constexpr int aev_region(int cap) { return cap > 64 ? cap : 64; }
__host__ __device__ constexpr bool aev_quads(int cap) { return cap <= 64; }

// NT: 16-block tiles of the angular one-hot (ceil(S (S + 1) / 2 / 16): one
// for up to five elements, two for six or seven, three for eight).
template <typename OutT, int NT, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Q > 1 ? 7 : 8, 8))) void k_aev_fwd(const int* __restrict__ dims, AevConst C,
                                                 const float4* __restrict__ rec,
                                                 const int2* __restrict__ counts, int cap,
                                                 const int* __restrict__ row_of,
                                                 OutT* __restrict__ out, int ld,
                                                 unsigned long long* __restrict__ kmask,
                                                 int sparse) {
  extern __shared__ float4 lds4[];
  const int n = dims[0];
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = lane_id();
  const int i0 = ((int)blockIdx.x * 4 + w) * Q;  // the wave's first atom
  if (i0 >= n) return;
  const int reg = aev_region(cap);
  float4* nd = lds4 + (size_t)w * reg;
  float2* nf0 = reinterpret_cast<float2*>(lds4 + (size_t)4 * reg);
  float2* nf = nf0 + (size_t)w * reg;
  int* nsp0 = reinterpret_cast<int*>(nf0 + (size_t)4 * reg);
  int* nsp = nsp0 + (size_t)w * reg;
  float* pw0 = reinterpret_cast<float*>(nsp0 + (size_t)4 * reg);  // [4][kPairChunk][8]
  float* pw = pw0 + w * kPairChunk * kNZ;
  float* pg0 = pw0 + 4 * kPairChunk * kNZ;                          // [4][kPairChunk][4]
  float* pg = pg0 + w * kPairChunk * kNA;
  int* pblk = reinterpret_cast<int*>(pg0 + 4 * kPairChunk * kNA) + w * kPairChunk;

  auto setup = [&](int slot, const float4 q, bool ang) __attribute__((always_inline)) {
    const float r = fast_sqrt(dist2(q.x, q.y, q.z));
    float dfr, dfa;
    const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
    const float fa = ang ? cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a) : 0.f;
    nd[slot] = make_float4(q.x, q.y, q.z, r);
    nf[slot] = make_float2(fr, fa);
    nsp[slot] = species_of(q);
  };

  // group g (lanes 16 g .. 16 g + 15) reads the counts and first 16 records
  // of atom i0 + g (one atom per wave: every group reads atom i0)
  const int g = Q > 1 ? lane >> 4 : 0, l = lane & 15;
  const int ig = i0 + g;
  const bool gin = ig < n;
  const float4 q0 = gin ? rec[(size_t)ig * cap + l] : make_float4(0.f, 0.f, 0.f, 0.f);
  const int2 cn = gin ? counts[ig] : make_int2(0, 0);
  const int nr_g = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na_g = cn.y < 0 ? 0 : (cn.y > nr_g ? nr_g : cn.y);
  const bool quad = Q > 1 && __ballot(nr_g > kQuadNbr) == 0;
  const int T_g = na_g * (na_g - 1) / 2;
  // quad waves with at most 16 pairs per atom: one pair table (slot 16 g + t)
  const bool joint = quad && __ballot(T_g > kQuadNbr) == 0;
  if (quad) {
    if (l < nr_g) setup(kQuadNbr * g + l, q0, l < na_g);
    wave_lds_sync();
    if (joint) {
      if (l < T_g)
        pair_geometry(l, na_g, C, nd + kQuadNbr * g, nf + kQuadNbr * g, nsp + kQuadNbr * g, pw, pg,
                      pblk, lane);
      wave_lds_sync();
    }
  }
  const int S = C.S;
  const int l16 = lane & 15, kq = lane >> 4;
  const float Rm = C.lane_tab[l16];
  const int z = l16 & 7, ah = l16 >> 3;
  const int nblk = S * (S + 1) / 2;

  for (int a = 0; a < Q; ++a) {
    const int i = i0 + a;
    if (i >= n) break;  // wave-uniform
    const int nr = __builtin_amdgcn_readlane(nr_g, kQuadNbr * a);
    const int na = __builtin_amdgcn_readlane(na_g, kQuadNbr * a);
    int base = kQuadNbr * a;
    if (!quad) {
      // this atom alone: every lane sets up its neighbors in slots [0, nr)
      base = 0;
      wave_lds_sync();  // the previous atom's passes have read the region
      const float4* arec = rec + (size_t)i * cap;
      for (int e = lane; e < nr; e += kWave) setup(e, arec[e], e < na);
      wave_lds_sync();
    }
    const float4* nda = nd + base;
    const float2* nfa = nf + base;
    const int* nspa = nsp + base;
    const int orow_i = row_of ? row_of[i] : i;
    OutT* orow = out + (size_t)orow_i * ld;
    // ---- radial: G[s][m] = sum over neighbors e of [species(e) == s] * term(e, m)
    // as MFMA products of a one-hot (species x 4 neighbors) with the terms
    // (4 neighbors x 16 shifts); lane (kq, l16) computes neighbor kq, shift l16.
    // With kmask, the lanes also count each element's neighbors (all, and
    // angular ones), which fixes the k-steps (32 feature columns)
    // holding a block this atom touches: the radial blocks of the elements
    // among its neighbors, the angular blocks of the element pairs among its
    // angular neighbors (a pair (a, a) needs two of them).  Every other
    // feature is zero, and the adjoint reads no dE/dG column outside them.
    unsigned long long kbits = ~0ull;
    unsigned sput = ~0u;
    {
      aev_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      float cnt = 0.f;  // lane (kq, l16): element l16 among entries kq, kq + 4, ...
      for (int e0 = 0; e0 < nr; e0 += 4) {
        const int e = e0 + kq;
        float term = 0.f, hot = 0.f;
        if (e < nr) {
          const float u = nda[e].w - Rm;
          term = C.cR * fast_exp2(-C.eta_r_l2e * u * u) * nfa[e].x;
          hot = nspa[e] == l16 ? 1.f : 0.f;
        }
        acc = mfma4(term, hot, acc);
        // (neighbors + 4096 x angular neighbors: exact, lists hold <= 512)
        cnt += (e < na ? 4097.f : 1.f) * hot;
      }
      if (kmask) {
        // the four entry groups' counts: lane l16 < S then holds element l16's
        cnt += __shfl_xor(cnt, 16, kWave);
        cnt += __shfl_xor(cnt, 32, kWave);
        const unsigned lm = (1u << S) - 1u;
        const unsigned rp = (unsigned)__ballot(cnt > 0.5f) & lm;
        const unsigned ap = (unsigned)__ballot(cnt > 4095.5f) & lm;
        const unsigned ad = (unsigned)__ballot(cnt > 8191.5f) & lm;
        // element x's row of the angular triangle, blocks (x, x + k), starts
        // at block x S - x (x - 1) / 2; (x, y > x) is touched when both
        // elements are among the angular neighbors, (x, x) when x is twice
        unsigned long long bm = 0;
        for (unsigned r = ap; r; r &= r - 1u) {
          const int x = __builtin_ctz(r);
          const unsigned row = (((ap >> x) & ~1u) | ((ad >> x) & 1u)) & ((1u << (S - x)) - 1u);
          bm |= (unsigned long long)row << (x * S - x * (x - 1) / 2);
        }
        const unsigned r2 = rp | (rp >> 1);  // k-step j holds elements 2j and 2j + 1
        const int k0 = C.A0 >> 5;  // block p spans k-step k0 + p (and k0 + p + 1 unaligned)
        kbits = (unsigned long long)((r2 & 1u) | ((r2 >> 1) & 2u) | ((r2 >> 2) & 4u) |
                                     ((r2 >> 3) & 8u)) |
                (bm << k0) | ((C.A0 & 31) ? bm << (k0 + 1) : 0ull);
        if (lane == 0) kmask[orow_i] = kbits;
        if (sparse) {
          // this lane's stores: bit 0 radial, bits 1 + 2 u and 2 + 2 u the
          // two halves of angular tile u (one k-step when A0 is aligned)
          sput = (unsigned)(kbits >> (l16 >> 1)) & 1u;
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            const int c = C.A0 + l16 * 32 + 4 * kq + 512 * u;
            const unsigned lo = (unsigned)(kbits >> (c >> 5)) & 1u;
            const unsigned hi =
                (C.A0 & 31) ? (unsigned)(kbits >> ((c + 16) >> 5)) & 1u : lo;
            sput |= (lo << (1 + 2 * u)) | (hi << (2 + 2 * u));
          }
        }
      }
      // (element slots from S up to the angular blocks are the gap: zero)
      if (l16 < (C.A0 >> 4) && (sput & 1u))
        Store<OutT>::put4(orow + l16 * kNR + 4 * kq, make_float4(acc[0], acc[1], acc[2], acc[3]));
    }

    // ---- angular: G[blk][a z] = sum over unordered pairs of angular
    // neighbors of [block(pair) == blk] * term(pair, a, z), four pairs per
    // pass.  Lane (kq, l16) takes pair kq and column l16 of each of the two
    // 16-column halves: angle shift z = l16 % 8 and radial shifts a = l16 / 8
    // and l16 / 8 + 2.  Tile u of the one-hot covers blocks 16 u .. 16 u + 15.
    {
      const int T = na * (na - 1) / 2;
      aev_f32x4 c0[NT], c1[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        c0[u] = aev_f32x4{0.f, 0.f, 0.f, 0.f};
        c1[u] = c0[u];
      }
      for (int p0 = 0; p0 < T; p0 += kPairChunk) {
        int tb = kQuadNbr * a;  // table slot of the chunk's first pair
        if (!joint) {
          tb = 0;
          wave_lds_sync();  // the previous chunk's passes have read the table
          if (p0 + lane < T) pair_geometry(p0 + lane, na, C, nda, nfa, nspa, pw, pg, pblk, lane);
          wave_lds_sync();
        }
        const int tn = T - p0 < kPairChunk ? T - p0 : kPairChunk;
        for (int t0 = 0; t0 < tn; t0 += 4) {
          const int t = t0 + kq;
          float b0 = 0.f, b1 = 0.f;
          int blk = -1;
          if (t < tn) {
            const int sl = tb + t;
            blk = pblk[sl];
            const float wz = pw[sl * kNZ + z];
            b0 = wz * pg[sl * kNA + ah];
            b1 = wz * pg[sl * kNA + ah + 2];
          }
          // a tile's products run only on passes that hold one of its blocks
          // (pairs come in species order, so most passes touch one tile)
#pragma unroll
          for (int u = 0; u < NT; ++u) {
            if (NT == 1 || __ballot(blk >= 16 * u && blk < 16 * u + 16) != 0) {
              const float hot = blk == l16 + 16 * u ? 1.f : 0.f;
              c0[u] = mfma4(b0, hot, c0[u]);
              c1[u] = mfma4(b1, hot, c1[u]);
            }
          }
        }
      }
      // column c of c0[u] is feature c of block 16 u + l16 (a = c / 8 for the
      // low radial shifts, z = c % 8); c1[u] holds features 16 + c
      OutT* ang = orow + C.A0 + l16 * 32 + 4 * kq;
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        if (l16 + 16 * u < nblk) {
          if (sput & (2u << (2 * u)))
            Store<OutT>::put4(ang + 512 * u, make_float4(c0[u][0], c0[u][1], c0[u][2], c0[u][3]));
          if (sput & (4u << (2 * u)))
            Store<OutT>::put4(ang + 512 * u + 16,
                              make_float4(c1[u][0], c1[u][1], c1[u][2], c1[u][3]));
        }
      }
    }
    for (int c = C.A0 + nblk * 32 + lane; c < ld; c += kWave) Store<OutT>::put(orow + c, 0.f);
  }
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

// Sixteen consecutive dE/dG values (one radial species block) as floats.
template <typename GT> struct Load16;
template <> struct Load16<float> {
  __device__ __forceinline__ static void get(const float* p, float (&v)[16]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 u = reinterpret_cast<const float4*>(p)[q];
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  }
};
template <> struct Load16<bf16_t> {
  __device__ __forceinline__ static void get(const bf16_t* p, float (&v)[16]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint4 u = reinterpret_cast<const uint4*>(p)[q];
      const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        v[8 * q + 2 * k] = __uint_as_float(w[k] << 16);
        v[8 * q + 2 * k + 1] = __uint_as_float(w[k] & 0xffff0000u);
      }
    }
  }
};

// The 32 dE/dG values of one angular pair block (four distance shifts x
// eight angle shifts, a-major), kept as loaded (BF16: two per register) and
// converted where used.
template <typename GT> struct Block32;
template <> struct Block32<float> {
  float v[32];
  __device__ __forceinline__ void load(const float* p) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 u = reinterpret_cast<const float4*>(p)[q];
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  }
  __device__ __forceinline__ float at(int k) const { return v[k]; }
};
template <> struct Block32<bf16_t> {
  unsigned w[16];
  __device__ __forceinline__ void load(const bf16_t* p) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 u = reinterpret_cast<const uint4*>(p)[q];
      w[4 * q] = u.x;
      w[4 * q + 1] = u.y;
      w[4 * q + 2] = u.z;
      w[4 * q + 3] = u.w;
    }
  }
  __device__ __forceinline__ float at(int k) const {
    return __uint_as_float((k & 1) ? (w[k >> 1] & 0xffff0000u) : (w[k >> 1] << 16));
  }
};

// One neighbor entry of the adjoint's LDS region: displacement and
// distance, cutoff values and derivatives, species.
__device__ __forceinline__ void adjoint_setup(int slot, const float4 q, bool ang,
                                              const AevConst& C, float4* nd, float4* nf,
                                              int* nsp) {
  const float r = fast_sqrt(dist2(q.x, q.y, q.z));
  float dfr, dfa = 0.f;
  const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
  const float fa = ang ? cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a) : 0.f;
  nd[slot] = make_float4(q.x, q.y, q.z, r);
  nf[slot] = make_float4(fr, fa, dfr, dfa);
  nsp[slot] = species_of(q);
}

// The radial and angular passes of one atom (nr neighbors, the first na
// angular, set up in nd, nf, nsp): dE/d(displacement) of every neighbor
// entry into grad (the radial pass stores, the angular pass adds).  The
// angular pass takes one of three forms (Mode):
//   kAngPairLanes: one lane per pair, 64 pairs per pass (long lists: the
//     pair's shared terms are computed once, not in eight lanes), and one
//     lane per neighbor entry in the radial pass;
//   kAngShiftLanes: eight lanes per pair (one per angle shift), eight pairs
//     per pass, fewer registers (the fallback of the four-atom kernels);
//   kAngShiftLanesOrdered: the same, adding the pass's eight pairs' terms one
//     pair after the other instead of with LDS atomics, so that every
//     entry's sum has a fixed order (deterministic mode).
constexpr int kAngPairLanes = 0, kAngShiftLanes = 1, kAngShiftLanesOrdered = 2;
template <typename GT, int Mode>
__device__ __forceinline__ void adjoint_passes(int nr, int na, const AevConst& C,
                                               const GT* __restrict__ grow, const float4* nd,
                                               const float4* nf, float4* grad, const int* nsp) {
  const int lane = lane_id();
  const int S = C.S;
  if constexpr (Mode == kAngPairLanes) {
    // ---- radial: one lane per neighbor entry, its 16 shifts against the 16
    // dE/dG values of its species block (two vector loads)
    for (int e = lane; e < nr; e += kWave) {
      const float4 v = nd[e];
      const float4 f = nf[e];
      float gv[16];
      Load16<GT>::get(grow + nsp[e] * kNR, gv);
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < kNR; ++m) {
        const float u = v.w - C.shf_r[m];
        acc += gv[m] * fast_exp2(-C.eta_r_l2e * u * u) * (f.z - C.eta_r2 * u * f.x);
      }
      const float sc = C.cR * acc * fast_rcp(v.w);
      grad[e] = make_float4(v.x * sc, v.y * sc, v.z * sc, 0.f);
    }
  } else
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

  if constexpr (Mode == kAngPairLanes) {
    // ---- angular: one lane per unordered pair (j, k), 64 pairs per pass.
    // What the pair's 32 terms share (cosine, sine, the four distance
    // Gaussians) is computed once; the lane walks the eight angle shifts and
    // contracts each with the pair block's dE/dG values (one vector load).
    const int T = na * (na - 1) / 2;
    const GT* gang = grow + C.A0;
    for (int t0 = 0; t0 < T; t0 += kWave) {
      // lanes past the last pair recompute it and add nothing
      const int t = t0 + lane;
      const bool valid = t < T;
      int ej, ek;
      decode_pair(valid ? t : T - 1, na, ej, ek);
      const float4 vj = nd[ej], vk = nd[ek];
      const float4 cj = nf[ej], ck = nf[ek];
      Block32<GT> gb;
      gb.load(gang + pair_block(nsp[ej], nsp[ek], S) * 32);
      const float fj = cj.y, fk = ck.y, dfj = cj.w, dfk = ck.w;
      const float rj = fast_rcp(vj.w), rk = fast_rcp(vk.w);
      const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) * (rj * rk);
      const float kc = C.kappa * cs;
      const float sn = fast_sqrt(fmaxf(1.f - kc * kc, 1e-12f));
      const float isn = fast_rcp(sn);
      const float dbar = 0.5f * (vj.w + vk.w);
      float e2[kNA], ue2[kNA];
#pragma unroll
      for (int a = 0; a < kNA; ++a) {
        const float u = dbar - C.shf_a[a];
        e2[a] = fast_exp2(-C.eta_a_l2e * u * u);
        ue2[a] = u * e2[a];
      }
      float X0 = 0.f, X1 = 0.f, Xc = 0.f;
#pragma unroll
      for (int z = 0; z < kNZ; ++z) {
        const float cz = C.lane_tab[kNR + z], sz = C.lane_tab[kNR + kNZ + z];
        float A0 = 0.f, A1 = 0.f;
#pragma unroll
        for (int a = 0; a < kNA; ++a) {
          A0 += gb.at(a * kNZ + z) * e2[a];
          A1 -= gb.at(a * kNZ + z) * ue2[a];
        }
        const float base_ = 0.5f + 0.5f * (kc * cz + sn * sz);
        const float pw = fast_exp2(C.zeta * fast_log2(base_));
        const float df1 = C.zeta * pw * fast_rcp(base_) * (C.kappa * (cz - kc * sz * isn));
        X0 += 2.f * pw * A0;
        X1 += 2.f * pw * A1;
        Xc += df1 * A0;
      }
      X1 *= C.eta_a;
      const float fcc = fj * fk;
      const float dEdc = Xc * fcc;
      const float dEdj = X1 * fcc + X0 * dfj * fk;
      const float dEdk = X1 * fcc + X0 * fj * dfk;
      const float aj = (dEdj - dEdc * cs * rj) * rj;
      const float ak = (dEdk - dEdc * cs * rk) * rk;
      const float bb = dEdc * rj * rk;
      // Entry j's terms: the pass's pairs of row j are consecutive lanes, so
      // a segmented sum over that run leaves the row's total in its last lane,
      // which adds it alone (LDS atomics on one address from up to 16 lanes
      // would serialize).  Lanes past the last pair lie after it.
      float sx = aj * vj.x + bb * vk.x, sy = aj * vj.y + bb * vk.y, sz = aj * vj.z + bb * vk.z;
      const int rs = (ej * (2 * na - ej - 1)) >> 1;  // the row's first pair
      const int s_lane = (rs > t0 ? rs : t0) - t0;
      const int re = rs + na - 2 - ej;               // and its last
      const int e_lane = (re < t0 + kWave - 1 ? re : t0 + kWave - 1) - t0;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const float ox = __shfl_up(sx, d, kWave), oy = __shfl_up(sy, d, kWave),
                    oz = __shfl_up(sz, d, kWave);
        if (lane - d >= s_lane) {
          sx += ox;
          sy += oy;
          sz += oz;
        }
      }
      if (lane == e_lane) {
        atomicAdd(&grad[ej].x, sx);
        atomicAdd(&grad[ej].y, sy);
        atomicAdd(&grad[ej].z, sz);
      }
      // entry k's terms: at most one per row, so few lanes share an entry
      if (valid) {
        atomicAdd(&grad[ek].x, ak * vk.x + bb * vj.x);
        atomicAdd(&grad[ek].y, ak * vk.y + bb * vj.y);
        atomicAdd(&grad[ek].z, ak * vk.z + bb * vj.z);
      }
    }
  } else
  // ---- angular: lanes (t, z), eight unordered pairs per pass
  {
    const int tz = lane & 7, tg = lane >> 3;
    const float cz = C.lane_tab[kNR + tz], sz = C.lane_tab[kNR + kNZ + tz];
    const float ra0 = C.shf_a[0], ra1 = C.shf_a[1], ra2 = C.shf_a[2], ra3 = C.shf_a[3];
    const int T = na * (na - 1) / 2;
    const GT* gang = grow + C.A0 + tz;
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
        if constexpr (Mode == kAngShiftLanes) {
          atomicAdd(&grad[ej].x, aj * vj.x + bb * vk.x);
          atomicAdd(&grad[ej].y, aj * vj.y + bb * vk.y);
          atomicAdd(&grad[ej].z, aj * vj.z + bb * vk.z);
          atomicAdd(&grad[ek].x, ak * vk.x + bb * vj.x);
          atomicAdd(&grad[ek].y, ak * vk.y + bb * vj.y);
          atomicAdd(&grad[ek].z, ak * vk.z + bb * vj.z);
        } else {
          for (int q = 0; q < 8; ++q) {
            if (tg == q) {
              float4 a = grad[ej];
              a.x += aj * vj.x + bb * vk.x;
              a.y += aj * vj.y + bb * vk.y;
              a.z += aj * vj.z + bb * vk.z;
              grad[ej] = a;
              float4 b = grad[ek];
              b.x += ak * vk.x + bb * vj.x;
              b.y += ak * vk.y + bb * vj.y;
              b.z += ak * vk.z + bb * vj.z;
              grad[ek] = b;
            }
            wave_lds_sync();
          }
        }
      }
    }
  }
  wave_lds_sync();
}

// The adjoint of atoms i0 .. i0 + 3, by one wave: dE/d(displacement) of every
// neighbor entry into the wave's LDS region (max(64, cap) entries of nd, nf,
// grad, nsp), then put(j, x, y, z) adds -sign * dE/dv to neighbor j and
// +sign * the sum to the centre atom.
//
// Quad waves (every atom with at most 16 neighbors) are built for latency:
// the adjoint waits on its gathers of dE/dG, so it issues as few dependent
// rounds of them as it can.  Lane (g, e) of group g sets up neighbor e of atom
// i0 + g and computes that neighbor's whole radial derivative (its 16 shifts
// against the 16 dE/dG values of its species block, two vector loads), so the
// radial part of all four atoms is one round; the angular pairs of the four
// atoms form one list that passes of eight pairs (eight lanes each) walk; the
// scatter and the centre sums (16-lane reductions) again take all four atoms
// at once.  Other waves take their atoms one at a time over the whole wave.
template <typename GT, int Q, typename Put>
__device__ __forceinline__ void adjoint_atoms(int i0, int n, const AevConst& C,
                                              const float4* __restrict__ rec,
                                              const int* __restrict__ nbr,
                                              const int2* __restrict__ counts, int cap,
                                              const int* __restrict__ row_of,
                                              const GT* __restrict__ g, int ldg, float sign,
                                              float4* nd, float4* nf, float4* grad, int* nsp,
                                              Put&& put) {
  const int lane = lane_id();
  // records, neighbor indices and counts of all four atoms are first-level
  // loads; group gq (lanes 16 gq .. 16 gq + 15) holds atom i0 + gq
  const int gq = Q > 1 ? lane >> 4 : 0, l = lane & 15;
  const int ig = i0 + gq;
  const bool gin = ig < n;
  const size_t gbase = (size_t)(gin ? ig : i0) * cap + l;
  const float4 q0 = gin ? rec[gbase] : make_float4(0.f, 0.f, 0.f, 0.f);
  const int2 cn = gin ? counts[ig] : make_int2(0, 0);
  const int nr_g = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na_g = cn.y < 0 ? 0 : (cn.y > nr_g ? nr_g : cn.y);
  const bool quad = Q > 1 && __ballot(nr_g > kQuadNbr) == 0;
  const int S = C.S;
  if (quad) {
    const int row_g = gin ? row_of[ig] : 0;
    // ---- setup and radial derivative, one lane per neighbor entry
    if (l < nr_g) {
      const float r = fast_sqrt(dist2(q0.x, q0.y, q0.z));
      float dfr, dfa = 0.f;
      const float fr = cutoff_val(r, C.inv_rc_r, dfr, C.pi_2rc_r);
      const float fa = l < na_g ? cutoff_val(r, C.inv_rc_a, dfa, C.pi_2rc_a) : 0.f;
      const int sp = species_of(q0);
      const int slot = kQuadNbr * gq + l;
      nd[slot] = make_float4(q0.x, q0.y, q0.z, r);
      nf[slot] = make_float4(fr, fa, dfr, dfa);
      nsp[slot] = sp;
      float gv[16];
      Load16<GT>::get(g + (size_t)row_g * ldg + sp * kNR, gv);
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < kNR; ++m) {
        const float u = r - C.shf_r[m];
        acc += gv[m] * fast_exp2(-C.eta_r_l2e * u * u) * (dfr - C.eta_r2 * u * fr);
      }
      const float sc = C.cR * acc * fast_rcp(r);
      grad[slot] = make_float4(q0.x * sc, q0.y * sc, q0.z * sc, 0.f);
    }
    wave_lds_sync();
    // ---- angular: the four atoms' pair lists as one list (pairs of atom a
    // from offset P_a), eight pairs per pass, lanes (pair tg, angle shift tz)
    const int na0 = __builtin_amdgcn_readlane(na_g, 0);
    const int na1 = __builtin_amdgcn_readlane(na_g, 16);
    const int na2 = __builtin_amdgcn_readlane(na_g, 32);
    const int na3 = __builtin_amdgcn_readlane(na_g, 48);
    const int P1 = na0 * (na0 - 1) / 2;
    const int P2 = P1 + na1 * (na1 - 1) / 2;
    const int P3 = P2 + na2 * (na2 - 1) / 2;
    const int Ttot = P3 + na3 * (na3 - 1) / 2;
    const int r0 = __builtin_amdgcn_readlane(row_g, 0);
    const int r1 = __builtin_amdgcn_readlane(row_g, 16);
    const int r2 = __builtin_amdgcn_readlane(row_g, 32);
    const int r3 = __builtin_amdgcn_readlane(row_g, 48);
    const int tz = lane & 7, tg = lane >> 3;
    const float cz = C.lane_tab[kNR + tz], sz = C.lane_tab[kNR + kNZ + tz];
    const float ra0 = C.shf_a[0], ra1 = C.shf_a[1], ra2 = C.shf_a[2], ra3 = C.shf_a[3];
    for (int t0 = 0; t0 < Ttot; t0 += 8) {
      // lanes past the last pair recompute it and contribute zero
      const int pt = t0 + tg;
      const bool valid = pt < Ttot;
      const int pc = valid ? pt : Ttot - 1;
      const int a = (pc >= P1) + (pc >= P2) + (pc >= P3);
      const int pa = a == 0 ? 0 : (a == 1 ? P1 : (a == 2 ? P2 : P3));
      const int na = a == 0 ? na0 : (a == 1 ? na1 : (a == 2 ? na2 : na3));
      const int ra = a == 0 ? r0 : (a == 1 ? r1 : (a == 2 ? r2 : r3));
      int ej, ek;
      decode_pair(pc - pa, na, ej, ek);
      ej += kQuadNbr * a;
      ek += kQuadNbr * a;
      const float4 vj = nd[ej], vk = nd[ek];
      const float4 cj = nf[ej], ck = nf[ek];
      const float fj = cj.y, fk = ck.y, dfj = cj.w, dfk = ck.w;
      const GT* gb = g + (size_t)ra * ldg + C.A0 + tz + pair_block(nsp[ej], nsp[ek], S) * 32;
      const float g0 = Store<GT>::get(gb), g1 = Store<GT>::get(gb + 8),
                  g2 = Store<GT>::get(gb + 16), g3 = Store<GT>::get(gb + 24);
      const float rj = fast_rcp(vj.w), rk = fast_rcp(vk.w);
      const float cs = (vj.x * vk.x + vj.y * vk.y + vj.z * vk.z) * (rj * rk);
      const float kc = C.kappa * cs;
      const float sn = fast_sqrt(fmaxf(1.f - kc * kc, 1e-12f));
      const float base_ = 0.5f + 0.5f * (kc * cz + sn * sz);
      const float pw = fast_exp2(C.zeta * fast_log2(base_));
      const float f1 = 2.f * pw;
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
    wave_lds_sync();
    // ---- scatter of all four atoms: neighbors get -sign * dE/dv, each
    // centre +sign * its group's sum
    float4 gv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l < nr_g) {
      gv = grad[kQuadNbr * gq + l];
      put(clampi(nbr[gbase], n), -sign * gv.x, -sign * gv.y, -sign * gv.z);
    }
    const float sx = group16_sum(gv.x), sy = group16_sum(gv.y), sz2 = group16_sum(gv.z);
    if (gin && l == 0) put(ig, sign * sx, sign * sy, sign * sz2);
    return;
  }
  for (int a = 0; a < Q; ++a) {
    const int i = i0 + a;
    if (i >= n) break;  // wave-uniform
    const int nr = __builtin_amdgcn_readlane(nr_g, kQuadNbr * a);
    const int na = __builtin_amdgcn_readlane(na_g, kQuadNbr * a);
    const GT* grow = g + (size_t)row_of[i] * ldg;
    // this atom alone over the whole wave
    const float4* arec = rec + (size_t)i * cap;
    const int* arow = nbr + (size_t)i * cap;
    // the scatter's first two rounds of neighbor indices, loaded now so that
    // their latency hides behind the passes
    const int j0 = lane < nr ? arow[lane] : 0;
    const int j1 = lane + kWave < nr ? arow[lane + kWave] : 0;
    for (int e = lane; e < nr; e += kWave) adjoint_setup(e, arec[e], e < na, C, nd, nf, nsp);
    wave_lds_sync();
    adjoint_passes<GT, Q == 1 ? kAngPairLanes : kAngShiftLanes>(nr, na, C, grow, nd, nf, grad,
                                                                nsp);
    float sx = 0.f, sy = 0.f, sz = 0.f;
    for (int e = lane; e < nr; e += kWave) {
      const float4 gv = grad[e];
      const int j = e < kWave ? j0 : (e < 2 * kWave ? j1 : arow[e]);
      put(clampi(j, n), -sign * gv.x, -sign * gv.y, -sign * gv.z);
      sx += gv.x;
      sy += gv.y;
      sz += gv.z;
    }
    sx = wave_sum_rows(sx);
    sy = wave_sum_rows(sy);
    sz = wave_sum_rows(sz);
    if (lane == 0) put(i, sign * sx, sign * sy, sign * sz);
    wave_lds_sync();  // the next atom reuses the region
  }
}

// Adjoint: g (rows of type GT, stride ldg) -> scatter into out (float32 [n][3]).
// sign = +1 writes forces (-dE/dr); sign = -1 writes the gradient dE/dr.
// With gidx, atom i's force goes to row gidx[i] of out ([n_total][3]; rows
// outside [0, n_total) are skipped; staging reports them).  Blocks from
// nb_adj on sum the molecular energies (one block per molecule), which need
// only the atomic energies of the forward pass: they fill the tail of the
// scatter instead of a launch of their own.
template <typename GT, int Q>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Q == 1 ? 6 : 4, 8))) void k_aev_bwd(
    const int* __restrict__ dims, AevConst C,
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
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int i0 = ((int)blockIdx.x * 4 + w) * Q;
  if (i0 >= n) return;
  const int reg = aev_region(cap);
  float4* nd = lds4 + (size_t)w * reg * 3;
  int* nsp = reinterpret_cast<int*>(lds4 + (size_t)4 * reg * 3) + w * reg;
  adjoint_atoms<GT, Q>(i0, n, C, rec, nbr, counts, cap, row_of, g, ldg, sign, nd, nd + reg,
                    nd + 2 * reg, nsp, [&](int j, float x, float y, float z) {
                      if (gidx) {
                        j = gidx[j];
                        if (j < 0 || j >= n_total) return;
                      }
                      unsafeAtomicAdd(out + 3 * j, x);
                      unsafeAtomicAdd(out + 3 * j + 1, y);
                      unsafeAtomicAdd(out + 3 * j + 2, z);
                    });
}

// Deterministic adjoint (gather mode): one atom per wave, as above, but the
// atom's dE/d(displacement) of every neighbor entry goes to pgrad[i * cap +
// e] instead of being scattered; a gather forms the forces from these rows
// (neighbors.hip).  Blocks from nb_adj on sum the molecular energies.
template <typename GT>
__global__ __launch_bounds__(256) void k_aev_bwd_det(const int* __restrict__ dims, AevConst C,
                                                     const float4* __restrict__ rec,
                                                     const int2* __restrict__ counts, int cap,
                                                     const int* __restrict__ row_of,
                                                     const GT* __restrict__ g, int ldg,
                                                     float4* __restrict__ pgrad, int nb_adj,
                                                     EnergyArgs EA) {
  extern __shared__ float4 lds4[];
  if ((int)blockIdx.x >= nb_adj) {  // block-uniform: the molecular energy sums
    energy_block((int)blockIdx.x - nb_adj, dims, EA);
    return;
  }
  const int n = dims[0];
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int i = (int)blockIdx.x * 4 + w;
  if (i >= n) return;
  const int lane = lane_id();
  const int reg = aev_region(cap);
  float4* nd = lds4 + (size_t)w * reg * 3;
  float4* nf = nd + reg;
  float4* grad = nd + 2 * reg;
  int* nsp = reinterpret_cast<int*>(lds4 + (size_t)4 * reg * 3) + w * reg;
  const int2 cn = counts[i];
  const int nr = cn.x < 0 ? 0 : (cn.x > cap ? cap : cn.x);
  const int na = cn.y < 0 ? 0 : (cn.y > nr ? nr : cn.y);
  const float4* arec = rec + (size_t)i * cap;
  for (int e = lane; e < nr; e += kWave) adjoint_setup(e, arec[e], e < na, C, nd, nf, nsp);
  wave_lds_sync();
  adjoint_passes<GT, kAngShiftLanesOrdered>(nr, na, C, g + (size_t)row_of[i] * ldg, nd, nf, grad,
                                            nsp);
  for (int e = lane; e < nr; e += kWave) pgrad[(size_t)i * cap + e] = grad[e];
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
template <typename GT, int Q>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_aev_bwd_mol(const int* __restrict__ dims, AevConst C,
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
  const int reg = aev_region(cap);
  float4* nd = lds4 + (size_t)w * reg * 3;
  int* nsp = reinterpret_cast<int*>(lds4 + (size_t)nw * reg * 3) + w * reg;
  float* win = reinterpret_cast<float*>(reinterpret_cast<int*>(lds4 + (size_t)nw * reg * 3) +
                                        (size_t)nw * reg);
  for (int t = threadIdx.x; t < 3 * kWin; t += blockDim.x) win[t] = 0.f;
  __syncthreads();
  for (int a = Q * w; a < kMolBlock; a += Q * nw) {
    const int i0 = base + a;
    if (i0 >= n) break;  // wave-uniform
    adjoint_atoms<GT, Q>(i0, n, C, rec, nbr, counts, cap, row_of, g, ldg, sign, nd, nd + reg,
                      nd + 2 * reg, nsp, [&](int j, float x, float y, float z) {
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
    wave_lds_sync();  // the next atoms reuse this wave's region
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

template <typename OutT, int Q>
static void launch_aev_fwd_q(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                             const int2* counts, int cap, const int* row_of, OutT* out, int ld,
                             unsigned long long* kmask, bool sparse, hipStream_t st) {
  const size_t lds = (size_t)4 * aev_region(cap) * kFwdBytesPerNbr +
                     (size_t)4 * kPairChunk * kFwdPairBytes;
  static const bool attr = (ensure_lds(k_aev_fwd<OutT, 1, Q>), ensure_lds(k_aev_fwd<OutT, 2, Q>),
                            ensure_lds(k_aev_fwd<OutT, 3, Q>), true);
  (void)attr;
  const int nblk = C.S * (C.S + 1) / 2;
  auto kern = nblk <= 16 ? k_aev_fwd<OutT, 1, Q>
                         : (nblk <= 32 ? k_aev_fwd<OutT, 2, Q> : k_aev_fwd<OutT, 3, Q>);
  const int per_block = 4 * Q;
  hipLaunchKernelGGL(kern, dim3((n_cap + per_block - 1) / per_block), dim3(256), lds, st, dims, C,
                     rec, counts, cap, row_of, out, ld, kmask, sparse ? 1 : 0);
}

template <typename OutT>
void launch_aev_fwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int2* counts, int cap, const int* row_of, OutT* out, int ld, bool det,
                    unsigned long long* kmask, bool sparse, hipStream_t st) {
  if (n_cap <= 0) return;
  sparse = sparse && kmask && ld <= 64 * 32;
  if (aev_quads(cap) && !det)
    launch_aev_fwd_q<OutT, 4>(dims, n_cap, C, rec, counts, cap, row_of, out, ld, kmask, sparse,
                              st);
  else
    launch_aev_fwd_q<OutT, 1>(dims, n_cap, C, rec, counts, cap, row_of, out, ld, kmask, sparse,
                              st);
}
template void launch_aev_fwd<float>(const int*, int, const AevConst&, const float4*, const int2*,
                                    int, const int*, float*, int, bool, unsigned long long*, bool,
                                    hipStream_t);
template void launch_aev_fwd<bf16_t>(const int*, int, const AevConst&, const float4*,
                                     const int2*, int, const int*, bf16_t*, int, bool,
                                     unsigned long long*, bool, hipStream_t);

template <typename GT, int Q>
static void launch_aev_bwd_q(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                             const int* nbr, const int2* counts, int cap, const int* row_of,
                             const GT* g, int ldg, float* out, float sign, const int* gidx,
                             int n_total, const int2* mrange, const EnergyArgs* energy,
                             int nmol_cap, hipStream_t st) {
  const int nb_e = energy && energy->E && nmol_cap > 0 ? nmol_cap : 0;
  const EnergyArgs ea = nb_e ? *energy : EnergyArgs{};
  if (mrange && !gidx) {
    // waves per workgroup: 8 while two workgroups fit a CU's LDS, else 4
    const int nw = cap <= 128 ? 8 : 4;
    const int nb_adj = n_cap > 0 ? (n_cap + kMolBlock - 1) / kMolBlock : 0;
    if (nb_adj + nb_e == 0) return;
    const size_t lds =
        (size_t)nw * aev_region(cap) * kBwdBytesPerNbr + (size_t)3 * kMolBlock * 3 * 4;
    static const bool attr = (ensure_lds(k_aev_bwd_mol<GT, Q>), true);
    (void)attr;
    hipLaunchKernelGGL((k_aev_bwd_mol<GT, Q>), dim3(nb_adj + nb_e), dim3(64 * nw), lds, st, dims,
                       C, rec, nbr, counts, cap, row_of, g, ldg, out, sign, mrange, nb_adj, ea);
    return;
  }
  const int nb_adj = n_cap > 0 ? (n_cap + 4 * Q - 1) / (4 * Q) : 0;
  if (nb_adj + nb_e == 0) return;
  const size_t lds = (size_t)4 * aev_region(cap) * kBwdBytesPerNbr;
  static const bool attr = (ensure_lds(k_aev_bwd<GT, Q>), true);
  (void)attr;
  hipLaunchKernelGGL((k_aev_bwd<GT, Q>), dim3(nb_adj + nb_e), dim3(256), lds, st, dims, C, rec,
                     nbr, counts, cap, row_of, g, ldg, out, sign, gidx, n_total, nb_adj, ea);
}

template <typename GT>
void launch_aev_bwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int* nbr, const int2* counts, int cap, const int* row_of, const GT* g,
                    int ldg, float* out, float sign, const int* gidx, int n_total,
                    const int2* mrange, const EnergyArgs* energy, int nmol_cap, float4* pgrad,
                    hipStream_t st) {
  if (pgrad) {
    const int nb_e = energy && energy->E && nmol_cap > 0 ? nmol_cap : 0;
    const EnergyArgs ea = nb_e ? *energy : EnergyArgs{};
    const int nb_adj = n_cap > 0 ? (n_cap + 3) / 4 : 0;
    if (nb_adj + nb_e == 0) return;
    const size_t lds = (size_t)4 * aev_region(cap) * kBwdBytesPerNbr;
    static const bool attr = (ensure_lds(k_aev_bwd_det<GT>), true);
    (void)attr;
    hipLaunchKernelGGL((k_aev_bwd_det<GT>), dim3(nb_adj + nb_e), dim3(256), lds, st, dims, C,
                       rec, counts, cap, row_of, g, ldg, pgrad, nb_adj, ea);
    return;
  }
  if (aev_quads(cap))
    launch_aev_bwd_q<GT, 4>(dims, n_cap, C, rec, nbr, counts, cap, row_of, g, ldg, out, sign,
                            gidx, n_total, mrange, energy, nmol_cap, st);
  else
    launch_aev_bwd_q<GT, 1>(dims, n_cap, C, rec, nbr, counts, cap, row_of, g, ldg, out, sign,
                            gidx, n_total, mrange, energy, nmol_cap, st);
}
template void launch_aev_bwd<float>(const int*, int, const AevConst&, const float4*, const int*,
                                    const int2*, int, const int*, const float*, int, float*, float,
                                    const int*, int, const int2*, const EnergyArgs*, int, float4*,
                                    hipStream_t);
template void launch_aev_bwd<bf16_t>(const int*, int, const AevConst&, const float4*, const int*,
                                     const int2*, int, const int*, const bf16_t*, int, float*,
                                     float, const int*, int, const int2*, const EnergyArgs*, int,
                                     float4*, hipStream_t);

}  // namespace nnp

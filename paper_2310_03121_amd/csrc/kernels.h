// Kernel entry points and launch helpers of the NNP engine.
#pragma once

#include "common.h"

namespace nnp {

enum { EPI_CELU = 0, EPI_HEAD = 1, EPI_BWD = 2, EPI_OUT = 3 };

struct GemmArgs {
  const void* A;
  int lda;
  const void* B;   // element s uses B + s * sB: [N][K] row-major, stride ldb
  const void* Bq;  // the same in MFMA fragment order (BF16; nullptr if absent)
  long sB;
  int ldb;
  const float* bias;
  int sBias;
  int N, K;
  const GroupTable* gt;
  void* C;
  int ldc;
  const void* H;   // EPI_BWD: activation whose CELU derivative scales acc
  int ldh;
  const float* w_out;  // EPI_HEAD: output-layer weights [S][N]
  int sWout;
  const float* b_out;  // [S]
  float* erow;         // [atoms] atomic energies in input atom order (EPI_HEAD)
  void* H3;            // optional store of the last hidden activation
  int ldh3;
  const int* perm;     // sorted row -> atom
  const int* mol;      // atom -> molecule
  const double* dLdE;  // per-molecule upstream gradient, or null for ones
  float* uprow;        // optional store of the per-row upstream gradient (EPI_HEAD)
  float alpha;
  float inv_alpha_l2e; // log2(e) / alpha
  float escale = 1.f;  // EPI_HEAD: factor on the upstream gradient (1 / ensemble size)
  // optional per-row k-step masks of the feature rows (launch_aev_fwd's
  // kmask; FP32 LDS-staged kernel): kmask_k skips the K stages (32 columns)
  // that every row of the tile has zero (layer 1, K = the feature columns);
  // kmask_n skips the column blocks no row of the tile needs (dE/dG: the
  // adjoint reads only a row's own k-steps)
  const unsigned long long* kmask_k = nullptr;
  const unsigned long long* kmask_n = nullptr;
};

struct MidArgs {
  const GroupTable* gt;
  const bf16_t* H1;               // [rows][W1]
  const bf16_t* W1;               // [S][W2][W1], fragment order
  const bf16_t* W2;               // [S][W3][W2], fragment order
  const bf16_t* W2T;              // [S][W2][W3], fragment order
  const bf16_t* W1T;              // [S][W1][W2], fragment order
  const float* b1;                // [S][W2]
  const float* b2;                // [S][W3]
  const float* wout;              // [S][W3]
  const float* bout;              // [S]
  float* erow;                    // [atoms] atomic energies, input atom order
  bf16_t* D1;                     // [rows][ld_d1], columns [0, W1)
  bf16_t* H2;                     // optional [rows][W2]
  bf16_t* H3;                     // optional [rows][W3]
  bf16_t* D3;                     // optional [rows][W3]
  bf16_t* D2;                     // optional [rows][W2]
  float* uprow;                   // optional [rows]
  const int* perm;
  const int* mol;
  const double* dLdE;
  float alpha;
  float inv_alpha_l2e;
  float escale = 1.f;             // factor on the upstream gradient (1 / ensemble size)
  int ld_d1 = 0;                  // row stride of D1 (0: W1)
  // the whole network per tile (k_mlp_net): layer 1 from X, dE/dG into G
  const bf16_t* X = nullptr;      // [rows][ldx] feature rows
  int ldx = 0;                    // row stride of X and G, layer 1's K (a multiple of 256)
  const bf16_t* W0 = nullptr;     // [S][W1][ldx], fragment order
  const float* b0 = nullptr;      // [S][W1]
  bf16_t* H1out = nullptr;        // [rows][W1]: H1, stored when D1 is (the weight gradients)
  const bf16_t* W0T = nullptr;    // [S][ldx][W1], fragment order
  bf16_t* G = nullptr;            // [rows][ldx] dE/dG, or null (no forces)
  // optional [rows]: per row, the k-steps (32 columns of X) that may be
  // nonzero (launch_aev_fwd's kmask); X is read, and G written, only there.
  // Null: every k-step (ldx <= 2048 either way).
  const unsigned long long* kmask = nullptr;
};

// Weight slots: member k of an ensemble, element s -> slot k * S + s.
struct PackArgs {
  const float* flat;
  long off[kMaxModels * kMaxS * kLayers];  // flat offset of W for (slot, layer)
  int S;                  // elements (slot = member * S + element)
  int n_models;
  float* WT0cf;           // ensembles: [S][F_pad][M * width1] member-concatenated W_0^T
  bf16_t* WT0cq;          // the same in MFMA fragment order (N = F_pad, K = M * width1)
  int width[kLayers + 1];
  int Fp;
  int r0, a0;             // layer 1: inputs from r0 on sit at columns from a0 on
  float* Wf[kLayers];     // W [slots][out][in_pad], row-major
  bf16_t* Wb[kLayers];
  float* WTf[kLayers];    // W^T [S][in_pad][out], row-major
  bf16_t* Wqb[kLayers];   // W in MFMA fragment order (N = out, K = in_pad)
  bf16_t* WTqb[kLayers];  // W^T in MFMA fragment order (N = in_pad, K = out)
  float* bias[kLayers];
  float* wout;
  float* bout;
};

struct EnergyArgs;  // energy_sum.h

// stage.hip
inline int stage_blocks(int n_cap) { return n_cap > 0 ? (n_cap + 255) / 256 : 1; }
// molecule offsets sampled into LDS by each staging block
constexpr int kOffSamples = 1024;
__global__ void k_fill_i32(int* p, int v, int n);
__global__ void k_fill_f32(float* p, float v, long n);
__global__ void k_fill_f64(double* p, double v, int n);
void launch_stage(int n_arg, int nmol_arg, int n_cap, int* dims, const float* pos,
                  const double* pos64, const int* gidx, int n_total, const int* species,
                  const int* off, int S, float4* xyzs, int* mol, int2* mrange, float* Fzero,
                  int* hist, uint32_t* status, bool clear_status,
                  int* zero, int nzero, hipStream_t st);
void launch_groups(const int* dims, int n_cap, int S, int* hist, GroupTable* gt, int* perm,
                   int rows_cap, const int* off, int wchunk_rows, uint32_t* status,
                   hipStream_t st);
// k_groups + k_scatter in one launch; for n_cap <= 256 * kFusedSortBlocks
constexpr int kFusedSortBlocks = 256;
void launch_sort_scatter(const int* dims, int n_cap, int S, const float4* xyzs, const int* hist,
                         GroupTable* gt, int* row, int* perm, int rows_cap, const int* off,
                         int wchunk_rows, uint32_t* status, hipStream_t st);
void launch_scatter(const int* dims, int n_cap, int S, const float4* xyzs, const int* hist,
                    int* row, int* perm, hipStream_t st);
void launch_energy(const int* dims, int nmol_cap, const int* off, const float4* xyzs,
                   const float* eatom, int n_models, long mstride, const double* eself,
                   double* E, uint32_t* status, hipStream_t st);
void launch_fill_i32(int* p, int v, int n, hipStream_t st);
void launch_fill_f32(float* p, float v, long n, hipStream_t st);
void launch_fill_f64(double* p, double v, int n, hipStream_t st);

// neighbors.hip
// Neighbor rows (ELL, row i at i * cap): nbr holds atom indices, rec the
// matching records (dx, dy, dz, species bits) with d = x_j - x_i (minimum
// image when periodic), computed by the cutoff predicate's own arithmetic.
void launch_pairs_mol(const int* dims, int n_cap, const AevConst& C, const float4* xyzs,
                      const int2* mrange, int cap, int* nbr, float4* rec, int2* counts,
                      uint32_t* status, hipStream_t st);
// launch_sort_scatter and launch_pairs_mol in one launch (n_cap <= 256 * kFusedSortBlocks)
void launch_sort_pairs_mol(const int* dims, int n_cap, int S, const int* hist, GroupTable* gt,
                           int* row, int* perm, int rows_cap, const int* off, int wchunk_rows,
                           const AevConst& C, const float4* xyzs, const int2* mrange, int cap,
                           int* nbr, float4* rec, int2* counts, uint32_t* status,
                           hipStream_t st);
// Periodic boxes: cell_cnt holds cell_zero_ints(ncell) ints that staging
// zeroed: the per-cell counts, then (up to kCellScanLds cells) the fill
// counters, or (more cells) the counting launch's done counter.
constexpr int kCellScanLds = 8192;
inline size_t cell_zero_ints(int ncell) {
  return ncell <= kCellScanLds ? 2 * (size_t)ncell : (size_t)ncell + 1;
}
void launch_pairs_cell(const int* dims, int n_cap, const AevConst& C, const BoxConst& B,
                       const float4* xyzs, int* cell_of, int* cell_cnt, int* cell_start,
                       int* cursor, int* cell_atoms, float4* cell_xyzs, int cap, int* nbr,
                       float4* rec, int2* counts, uint32_t* status, hipStream_t st);
// Deterministic forces from the adjoint's per-entry rows pgrad ([n][cap],
// dE_i/d(displacement of entry e)): atom a's row out[gidx ? gidx[a] : a] +=
// sign * sum over a's entries e, in list order, of pgrad[a][e] -
// pgrad[j_e][slot of a in j_e's list] (the lists are symmetric; the slot is
// found by binary search on the sort key).  One wave per atom; each row is
// added to once (no atomics).
void launch_force_gather(const int* dims, int n_cap, const float4* xyzs, const float4* rec,
                         const int* nbr, const int2* counts, int cap, const float4* pgrad,
                         float* out, float sign, const int* gidx, int n_total, hipStream_t st);

// aev.hip
// det: one atom per wave whatever the capacity (the order of every sum is
// then a function of the atom's own list only).  kmask (optional, [rows]):
// per row, bit q set when k-step q (feature columns 32 q .. 32 q + 31) holds
// a block the atom touches; sparse (needs kmask and ld <= 2048): only those
// k-steps of the row are stored (the rest of the row is left as it was).
template <typename OutT>
void launch_aev_fwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int2* counts, int cap, const int* row_of, OutT* out, int ld, bool det,
                    unsigned long long* kmask, bool sparse, hipStream_t st);
// pgrad: the deterministic adjoint, writing per-entry rows to pgrad (the
// caller then runs launch_force_gather) instead of scattering into out
template <typename GT>
void launch_aev_bwd(const int* dims, int n_cap, const AevConst& C, const float4* rec,
                    const int* nbr, const int2* counts, int cap, const int* row_of, const GT* g,
                    int ldg, float* out, float sign, const int* gidx, int n_total,
                    const int2* mrange, const EnergyArgs* energy, int nmol_cap, float4* pgrad,
                    hipStream_t st);

// mlp.hip
template <typename T>
bool launch_gemm(int epi, const GemmArgs& a, int rows_cap, hipStream_t st);
// Weight gradients of all layers (input layer first): per-chunk partials in
// one launch (plus one per layer whose widths the MFMA tiles do not take),
// then the chunk-ordered sum into dparams[param_off_dev[s] + e], e over the
// element's whole flat parameter vector.  partial holds n_chunks_cap times
// that vector's length in floats.
struct WgradLayer {
  const void* D;  // [rows][ldd] adjoint of the layer's output
  const void* H;  // [rows][ldh] the layer's input
  int ldd, ldh, Nout, Nin;
  bool d_fp32;    // D is FP32 (the output layer's), else the operand type
  // input i (of Nin, in the parameters' order) is column i of H, or
  // i + hgap from hgap0 on (the feature rows' gap before the angular blocks)
  int hgap0 = 1 << 30, hgap = 0;
};
template <typename T>
void launch_wgrad_net(const GroupTable* gt, int S, int n_chunks_cap, int chunk,
                      const WgradLayer* layers, int n_layers, float* partial, float* dparams,
                      const long* param_off_dev, hipStream_t st);
void launch_pack(const PackArgs& p, int slots, hipStream_t st);

// mlp_mid.hip
bool launch_mlp_mid(const int* width, const MidArgs& a, int rows_cap, hipStream_t st);
// Layer 1, the fused middle and dE/dG in one launch (one workgroup per
// 128-row tile; H1 and D1 stay in LDS).  Widths 1008-256-192-160 with a
// padded feature count that is a multiple of 256; returns false otherwise.
bool launch_mlp_net(const int* width, const MidArgs& a, int rows_cap, hipStream_t st);

// md.hip
void launch_vv_kick_drift(const int* dims, int n_cap, double* x, double* v, const float* F,
                          const double* mass, double dt, float* pos32, hipStream_t st);
void launch_vv_kick(const int* dims, int n_cap, double* v, const float* F, const double* mass,
                    double dt, hipStream_t st);
void launch_lfm_step(const int* dims, int n_cap, double* x, double* v, const float* F,
                     const double* mass, double dt, double c, double kT_acc, uint64_t seed,
                     uint64_t step, float* pos32, hipStream_t st);
void launch_serve_lfm(const int* dims, int n_cap, const int* mol, const int* off,
                      const int* kdone, const int* nsteps, const uint64_t* seed, double* x,
                      double* v, const float* F, const double* mass, double dt, double c,
                      double kT_acc, hipStream_t st);
void launch_kinetic(const int* dims, int nmol_cap, const int* off, const double* v,
                    const double* mass, double* ke, int* kdone, hipStream_t st);
void launch_gather_rows(const int* src, int n, const double* x_old, const double* v_old,
                        const int* sp_old, const double* m_old, const float* f_old,
                        const double* x_new_in, const double* v_new_in, const int* sp_new_in,
                        const double* m_new_in, double* x, double* v, int* sp, double* m, float* f,
                        hipStream_t st);
void launch_serve_integrate(const int* dims, int n_cap, const int* mol, const int* kdone,
                            const int* nsteps, double* x, double* v, const float* F,
                            const double* mass, double dt, hipStream_t st);


}  // namespace nnp

// Host side of the NNP engine: the C ABI declared in include/nnp.h.
//
// A handle holds the symmetry-function constants and the packed per-element
// weights on one device.  An evaluation carves the caller's workspace,
// enqueues the kernels of the path on the caller's stream and returns:
//   stage + species sort -> neighbor search -> symmetry functions ->
//   network layers (grouped GEMMs) -> FP64 energy sums ->
//   adjoint layers -> symmetry-function adjoint + force scatter.
// Nothing here synchronises except nnp_check and the server's retire step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/nnp.h"
#include "kernels.h"
#include "energy_sum.h"

using namespace nnp;

struct nnp_handle {
  int device = 0;
  nnp_precision prec = NNP_MLP_FP32;
  AevConst C{};
  int S = 0, F = 0, Fp = 0;
  int width[kLayers + 1] = {};
  float alpha = 0.1f;
  int max_nbr = 128;
  bool triclinic = false;               // box arguments are 9 floats (cell rows)
  bool deterministic = false;           // forces by gather (no floating-point atomics)
  int n_models = 1;                     // ensemble members (weight slot = member * S + element)
  size_t n_params = 0;                  // all members
  long param_off[kMaxModels * kMaxS][kLayers] = {};  // flat offset of W for (slot, layer)
  char* dmem = nullptr;
  float* flat = nullptr;
  float* Wf[kLayers] = {};     // row-major W and W^T (LDS-staged kernels)
  bf16_t* Wb[kLayers] = {};
  float* WTf[kLayers] = {};
  bf16_t* Wqb[kLayers] = {};   // fragment order, W and W^T (BF16 body kernels)
  bf16_t* WTqb[kLayers] = {};
  float* bias[kLayers] = {};
  float* WT0cf = nullptr;      // ensembles: member-concatenated W_0^T (dE/dG in one product)
  bf16_t* WT0cq = nullptr;
  float* wout = nullptr;
  float* bout = nullptr;
  double* eself = nullptr;
  long* param_off_dev = nullptr;  // [kLayers][S]
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;        // reusable events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  size_t ev_next = 0;
  double prof_ms[32] = {};
  long long prof_n[32] = {};
};

// Workspace of the allocation-free entry point (nnp_energy_forces_noalloc):
// one evaluation's workspace of at most kScratchBytes, held by every device
// the library runs on until the process ends.  On the host the name stands
// in for the symbol and is not a device address: host code uses only the
// per-device address that scratch_ptr() looks up.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kWChunk = 1024;  // rows per weight-gradient partial

// Device address of `scratch` on device `dev`: looked up once per device
// (with that device current) by hipGetSymbolAddress, then cached.  Returns
// null when the lookup fails.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// Owned/ghost evaluation: group offsets {0, n_owned, n} and upstream {1, 0}.
__global__ void k_owned_groups(int n, int n_owned, int* __restrict__ off,
                               double* __restrict__ up) {
  if (threadIdx.x == 0) {
    off[0] = 0;
    off[1] = n_owned;
    off[2] = n;
    up[0] = 1.0;
    up[1] = 0.0;
  }
}

// Copies the evaluation's status word to the caller (one thread).
__global__ void k_copy_status(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

enum Stage {
  ST_STAGE = 0, ST_PAIRS, ST_AEV, ST_L1, ST_L2, ST_HEAD, ST_ENERGY, ST_BWD3, ST_BWD2, ST_GRADG,
  ST_AEVBWD, ST_WGRAD, ST_MID, ST_NET, ST_COUNT
};
const char* kStageNames[ST_COUNT] = {
    "stage+sort", "neighbors", "aev_fwd", "mlp_layer1", "mlp_layer2", "mlp_layer3_head",
    "energy_sum", "mlp_bwd_layer3", "mlp_bwd_layer2", "mlp_bwd_dEdG", "aev_bwd_forces",
    "weight_grads", "mlp_mid_fused", "mlp_net_fused"};

hipEvent_t prof_event(nnp_handle* h) {
  if (h->ev_next == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_next++];
}

// Records an event pair around one stage when profiling is enabled.
struct StageTimer {
  nnp_handle* h;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(nnp_handle* h_, bool on, int s, hipStream_t st_) : h(h_), stage(s), st(st_) {
    if (on && h->prof && (a = prof_event(h))) (void)hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = prof_event(h);
    if (!b) return;
    (void)hipEventRecord(b, st);
    h->ev_pending.push_back({stage, {a, b}});
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Plan {
  int n = 0, nmol = 0, rows_cap = 0, cap = 0, nblk = 0, nwchunks = 0;
  BoxConst B{};
  int ncell = 0;
  size_t total = 0;
  size_t status, dims, gt, xyzs, mol, mrange, row, perm, hist, nbr, counts, rec;
  size_t cell_of, cell_cnt, cell_start, cursor, cell_atoms, cell_xyzs;
  size_t X, H1, H2, H3, D3, D2, D1, G, erow, uprow, wpart, pos32;
  size_t kmask;  // per feature row: the k-steps that may be nonzero
  size_t pgrad;  // deterministic mode: per-entry adjoint rows [n][cap]
  size_t grp;    // owned/ghost evaluation: group offsets (3 int) and upstream (2 double)
};

bool make_box(const nnp_handle* h, const float* box, BoxConst& B) {
  B = BoxConst{};
  if (!box) {
    for (int d = 0; d < 3; ++d) {
      B.L[d] = 1.f;
      B.invL[d] = 1.f;
      B.nc[d] = 1;
      B.cell_scale[d] = 1.f;
    }
    return true;
  }
  const float rc = 1.f / h->C.inv_rc_r;
  if (h->triclinic) {
    // rows a, b, c of a reduced cell; cells are binned along the fractional
    // coordinates, sized by the perpendicular widths
    B.periodic = 2;
    double v[3][3];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        if (!std::isfinite(box[3 * r + q])) return false;
        v[r][q] = box[3 * r + q];
        B.v[r][q] = box[3 * r + q];
      }
    if (v[0][1] != 0.0 || v[0][2] != 0.0 || v[1][2] != 0.0) return false;
    if (!(v[0][0] > 0.0 && v[1][1] > 0.0 && v[2][2] > 0.0)) return false;
    if (std::fabs(v[1][0]) > 0.5 * v[0][0] || std::fabs(v[2][0]) > 0.5 * v[0][0] ||
        std::fabs(v[2][1]) > 0.5 * v[1][1])
      return false;
    auto cross_norm = [&](int p, int q) {
      const double x = v[p][1] * v[q][2] - v[p][2] * v[q][1];
      const double y = v[p][2] * v[q][0] - v[p][0] * v[q][2];
      const double z = v[p][0] * v[q][1] - v[p][1] * v[q][0];
      return std::sqrt(x * x + y * y + z * z);
    };
    const double vol = v[0][0] * v[1][1] * v[2][2];
    const double wd[3] = {vol / cross_norm(1, 2), vol / cross_norm(2, 0), vol / cross_norm(0, 1)};
    for (int d = 0; d < 3; ++d) {
      if (!(wd[d] >= 2.0 * rc)) return false;
      int nc = (int)std::floor(wd[d] / ((double)rc + 1e-3));
      if (nc < 3) nc = 1;
      if (nc > 128) nc = 128;
      B.nc[d] = nc;
      B.L[d] = (float)v[d][d];
      B.invL[d] = 1.0f / B.v[d][d];
      B.inv_diag[d] = 1.0f / B.v[d][d];
      B.cell_scale[d] = (float)nc;
    }
    return true;
  }
  B.periodic = 1;
  for (int d = 0; d < 3; ++d) {
    const float L = box[d];
    if (!(L >= 2.f * rc) || !std::isfinite(L)) return false;
    B.L[d] = L;
    B.invL[d] = 1.0f / L;
    int nc = (int)std::floor((double)L / ((double)rc + 1e-3));
    if (nc < 3) nc = 1;
    if (nc > 128) nc = 128;
    B.nc[d] = nc;
    B.cell_scale[d] = (float)nc / L;
  }
  return true;
}

// wgrad = false leaves out the weight-gradient partials (calls that never ask
// for parameter gradients).
Plan make_plan(const nnp_handle* h, int n, int nmol, const BoxConst& B, bool wgrad = true) {
  Plan P;
  P.n = n;
  P.nmol = nmol;
  P.cap = h->max_nbr;
  P.B = B;
  P.ncell = B.periodic ? B.nc[0] * B.nc[1] * B.nc[2] : 0;
  P.rows_cap = (int)align_up((size_t)std::max(n, 1), kPad) + h->S * kPad;
  P.nblk = stage_blocks(n);
  P.nwchunks = (n + kWChunk - 1) / kWChunk + h->S;
  const size_t esz = h->prec == NNP_MLP_BF16 ? 2 : 4;
  const size_t R = (size_t)P.rows_cap;
  const size_t N = (size_t)std::max(n, 1);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max(bytes, (size_t)1), 256);
    return at;
  };
  P.status = take(16);
  P.dims = take(16);
  P.gt = take(sizeof(GroupTable));
  P.xyzs = take(N * 16);
  P.mol = take(N * 4);
  P.row = take(N * 4);
  P.perm = take(R * 4);
  P.hist = take((size_t)(kMaxS + 1) * P.nblk * 4);
  P.nbr = take(N * P.cap * 4);
  P.counts = take(N * 8);
  P.rec = take(N * P.cap * 16);
  P.pgrad = h->deterministic ? take(N * P.cap * 16) : 0;
  P.grp = take(64);
  if (B.periodic) {
    P.cell_of = take(N * 4);
    P.cell_cnt = take(cell_zero_ints(P.ncell) * 4);  // counts and binning counters (zeroed)
    P.cell_start = take((size_t)(P.ncell + 1) * 4);
    P.cursor = take((size_t)P.ncell * 4);
    P.cell_atoms = take(N * 4);
    P.cell_xyzs = take(N * 16);
    P.mrange = 0;
  } else {
    P.mrange = take(N * 8);
    P.cell_of = P.cell_cnt = P.cell_start = P.cursor = P.cell_atoms = P.cell_xyzs = 0;
  }
  const int w1 = h->width[1], w2 = h->width[2], w3 = h->width[3];
  P.X = take(R * h->Fp * esz);
  P.kmask = take(R * 8);
  P.H1 = take(R * w1 * esz);
  P.H2 = take(R * w2 * esz);
  P.H3 = take(R * w3 * esz);
  P.D3 = take(R * w3 * esz);
  P.D2 = take(R * w2 * esz);
  P.D1 = take(R * w1 * h->n_models * esz);  // members side by side in each row
  P.G = take(R * h->Fp * esz);
  P.erow = take(R * 4 * h->n_models);
  P.uprow = take(R * 4);
  size_t plen = 0;  // one element's parameters
  for (int l = 0; l < kLayers; ++l) {
    const size_t in = l == 0 ? h->F : h->width[l];
    plen += (size_t)h->width[l + 1] * in + h->width[l + 1];
  }
  P.wpart = wgrad ? take((size_t)P.nwchunks * plen * 4) : 0;
  P.pos32 = take(N * 12);
  P.total = o;
  return P;
}

template <typename T> T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

bool hip_ok(hipError_t e) { return e == hipSuccess; }

// The launches of this call succeeded: the runtime's last error is clear.
// hipErrorNotReady is no failure: the runtime also records it as the last
// error when an event or stream query (the serving loop's, or the caller's)
// finds work still running, and it would otherwise fail the next call.
bool launches_ok() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess || e == hipErrorNotReady;
}

// ---------------------------------------------------------------- the path

struct EvalIO {
  int n_arg, nmol_arg;  // >= 0: counts passed by value; -1: read from the workspace
  const float* pos;     // float32 positions, or
  const double* pos64;  // float64 positions (MD state), rounded to float32 on staging
  const int* species;
  const int* off;
  double* E;            // may be null
  float* out3;          // forces (sign +1) or dL/dpos (sign -1), may be null
  float sign;
  const double* dLdE;   // null: unit upstream
  float* dparams;       // weight gradients, may be null
  const int* gidx = nullptr;  // subset mode: rows of pos and out3 ([n_total][3]) per atom;
  int n_total = 0;            // forces are added to out3, not stored
  bool timed = true;          // stage events when profiling (they may create events)
  bool keep_status = false;   // OR into the status word instead of clearing it first
};

template <typename T>
nnp_status run_path(nnp_handle* h, const Plan& P, void* ws, const EvalIO& io, hipStream_t st) {
  int* dims = at<int>(ws, P.dims);
  uint32_t* status = at<uint32_t>(ws, P.status);
  GroupTable* gt = at<GroupTable>(ws, P.gt);
  float4* xyzs = at<float4>(ws, P.xyzs);
  int* mol = at<int>(ws, P.mol);
  int2* mrange = P.mrange ? at<int2>(ws, P.mrange) : nullptr;
  int* row = at<int>(ws, P.row);
  int* perm = at<int>(ws, P.perm);
  int* hist = at<int>(ws, P.hist);
  int* nbr = at<int>(ws, P.nbr);
  int2* counts = at<int2>(ws, P.counts);
  float4* rec = at<float4>(ws, P.rec);
  const int S = h->S, Fp = h->Fp;
  const int w1 = h->width[1], w2 = h->width[2], w3 = h->width[3];
  const bool bf = h->prec == NNP_MLP_BF16;
  const bool need_bwd = io.out3 || io.dparams;

  {
    StageTimer t(h, io.timed, ST_STAGE, st);
    launch_stage(io.n_arg, io.nmol_arg, P.n, dims, io.pos, io.pos64, io.gidx, io.n_total,
                 io.species, io.off, S, xyzs, mol, mrange, io.gidx ? nullptr : io.out3, hist,
                 status, !io.keep_status, P.B.periodic ? at<int>(ws, P.cell_cnt) : nullptr,
                 P.B.periodic ? cell_zero_ints(P.ncell) : 0, st);
    if (P.nblk > kFusedSortBlocks) {
      launch_groups(dims, P.n, S, hist, gt, perm, P.rows_cap, io.off, kWChunk, status, st);
      launch_scatter(dims, P.n, S, xyzs, hist, row, perm, st);
    } else if (P.B.periodic) {
      launch_sort_scatter(dims, P.n, S, xyzs, hist, gt, row, perm, P.rows_cap, io.off, kWChunk,
                          status, st);
    }
  }
  {
    StageTimer t(h, io.timed, ST_PAIRS, st);
    if (!P.B.periodic && P.nblk <= kFusedSortBlocks) {
      // molecules: the sort and the pair scan share one launch
      launch_sort_pairs_mol(dims, P.n, S, hist, gt, row, perm, P.rows_cap, io.off, kWChunk,
                            h->C, xyzs, mrange, P.cap, nbr, rec, counts, status, st);
    } else if (P.B.periodic) {
      launch_pairs_cell(dims, P.n, h->C, P.B, xyzs, at<int>(ws, P.cell_of),
                        at<int>(ws, P.cell_cnt), at<int>(ws, P.cell_start),
                        at<int>(ws, P.cursor), at<int>(ws, P.cell_atoms),
                        at<float4>(ws, P.cell_xyzs), P.cap, nbr, rec, counts, status, st);
    } else {
      launch_pairs_mol(dims, P.n, h->C, xyzs, mrange, P.cap, nbr, rec, counts, status, st);
    }
  }
  T* X = at<T>(ws, P.X);
  unsigned long long* kmask = at<unsigned long long>(ws, P.kmask);
  // BF16 with gradients, one network: layer 1, the fused middle and dE/dG
  // in one launch per tile (H1 and D1 stay in LDS)
  const bool net_path = bf && need_bwd && h->n_models == 1 && h->width[1] == 256 &&
                        h->width[2] == 192 && h->width[3] == 160 && Fp % 256 == 0 &&
                        Fp <= 2048;
  {
    StageTimer t(h, io.timed, ST_AEV, st);
    // the whole-network kernel reads each row's own k-steps only; the weight
    // gradients and the layer kernels read whole rows
    launch_aev_fwd<T>(dims, P.n, h->C, rec, counts, P.cap, row, X, Fp, h->deterministic, kmask,
                      net_path && !io.dparams, st);
  }

  T* H1 = at<T>(ws, P.H1);
  T* H2 = at<T>(ws, P.H2);
  T* H3 = at<T>(ws, P.H3);
  T* D3 = at<T>(ws, P.D3);
  T* D2 = at<T>(ws, P.D2);
  T* D1 = at<T>(ws, P.D1);
  T* G = at<T>(ws, P.G);
  float* erow = at<float>(ws, P.erow);
  // B operands: row-major W (both precisions) and W^T (FP32), and the BF16
  // fragment-order copies of W and W^T
  const void* W[kLayers];
  const void* WT[kLayers];
  const void* Wq[kLayers];
  const void* WTq[kLayers];
  for (int l = 0; l < kLayers; ++l) {
    W[l] = bf ? (const void*)h->Wb[l] : (const void*)h->Wf[l];
    WT[l] = bf ? nullptr : (const void*)h->WTf[l];
    Wq[l] = bf ? (const void*)h->Wqb[l] : nullptr;
    WTq[l] = bf ? (const void*)h->WTqb[l] : nullptr;
  }
  const int M = h->n_models;
  const int ldd1 = M * w1;  // D1 row: the members' delta1 side by side
  const float escale = 1.f / (float)M;
  const size_t esz = sizeof(T);
  bool ok = true;
  bool net_fused = false;  // the whole network ran as one launch (dE/dG included)
  for (int k = 0; k < M; ++k) {
    // member k: weight slots k * S .. k * S + S - 1
    const int q0 = k * S;
    float* erow_k = erow + (size_t)k * P.rows_cap;
    T* D1k = D1 + (size_t)k * w1;
    const void* Wk[kLayers];
    const void* WTk[kLayers];
    const void* Wqk[kLayers];
    const void* WTqk[kLayers];
    for (int l = 0; l < kLayers - 1; ++l) {
      const size_t inp = l == 0 ? (size_t)Fp : (size_t)h->width[l];
      const size_t slot = (size_t)h->width[l + 1] * inp;  // elements per weight slot
      Wk[l] = W[l] ? (const char*)W[l] + q0 * slot * esz : nullptr;
      WTk[l] = WT[l] ? (const char*)WT[l] + q0 * slot * esz : nullptr;
      Wqk[l] = Wq[l] ? (const char*)Wq[l] + q0 * slot * esz : nullptr;
      WTqk[l] = WTq[l] ? (const char*)WTq[l] + q0 * slot * esz : nullptr;
    }
    const float* bias_k[kLayers - 1];
    for (int l = 0; l < kLayers - 1; ++l) bias_k[l] = h->bias[l] + (size_t)q0 * h->width[l + 1];
    const float* wout_k = h->wout + (size_t)q0 * w3;
    const float* bout_k = h->bout + q0;
    if (net_path) {
      MidArgs ma{};
      ma.gt = gt;
      ma.W1 = static_cast<const bf16_t*>(Wqk[1]);
      ma.W2 = static_cast<const bf16_t*>(Wqk[2]);
      ma.W2T = static_cast<const bf16_t*>(WTqk[2]);
      ma.W1T = static_cast<const bf16_t*>(WTqk[1]);
      ma.b1 = bias_k[1];
      ma.b2 = bias_k[2];
      ma.wout = wout_k;
      ma.bout = bout_k;
      ma.erow = erow_k;
      ma.D1 = io.dparams ? reinterpret_cast<bf16_t*>(D1k) : nullptr;  // the weight gradients' copy
      ma.ld_d1 = ldd1;
      ma.escale = escale;
      if (io.dparams) {
        ma.H2 = reinterpret_cast<bf16_t*>(H2);
        ma.H3 = reinterpret_cast<bf16_t*>(H3);
        ma.D3 = reinterpret_cast<bf16_t*>(D3);
        ma.D2 = reinterpret_cast<bf16_t*>(D2);
        ma.uprow = at<float>(ws, P.uprow);
      }
      ma.perm = perm;
      ma.mol = mol;
      ma.dLdE = io.dLdE;
      ma.alpha = h->alpha;
      ma.inv_alpha_l2e = (float)(1.4426950408889634 / h->alpha);
      ma.X = reinterpret_cast<const bf16_t*>(X);
      ma.ldx = Fp;
      ma.W0 = static_cast<const bf16_t*>(Wqk[0]);
      ma.b0 = bias_k[0];
      ma.H1out = reinterpret_cast<bf16_t*>(H1);
      ma.W0T = static_cast<const bf16_t*>(WTq[0]);
      ma.G = io.out3 ? reinterpret_cast<bf16_t*>(G) : nullptr;
      ma.kmask = kmask;
      StageTimer t(h, io.timed, ST_NET, st);
      // (the feature rows may be stored sparse: no other kernel may take over)
      ok &= launch_mlp_net(h->width, ma, P.rows_cap, st);
      net_fused = true;
      continue;
    }
    GemmArgs g{};
    g.gt = gt;
    g.alpha = h->alpha;
    g.inv_alpha_l2e = (float)(1.4426950408889634 / h->alpha);
    g.escale = escale;
    // layer 1: H1 = CELU(X W0^T + b0)
    g.A = X; g.lda = Fp; g.B = Wk[0]; g.Bq = Wqk[0]; g.sB = (long)w1 * Fp; g.ldb = Fp;
    g.bias = bias_k[0]; g.sBias = w1; g.N = w1; g.K = Fp; g.C = H1; g.ldc = w1;
    g.kmask_k = kmask;  // (whole rows here: skipped stages are all zero)
    {
      StageTimer t(h, io.timed, ST_L1, st);
      ok &= launch_gemm<T>(EPI_CELU, g, P.rows_cap, st);
    }
    g.kmask_k = nullptr;
    // BF16 with gradients: one fused launch for layer 2, the energy head and the
    // adjoint of layers 3 and 2 (intermediates stay in LDS)
    bool fused = false;
    if (bf && need_bwd) {
      MidArgs ma{};
      ma.gt = gt;
      ma.H1 = reinterpret_cast<const bf16_t*>(H1);
      ma.W1 = static_cast<const bf16_t*>(Wqk[1]);
      ma.W2 = static_cast<const bf16_t*>(Wqk[2]);
      ma.W2T = static_cast<const bf16_t*>(WTqk[2]);
      ma.W1T = static_cast<const bf16_t*>(WTqk[1]);
      ma.b1 = bias_k[1];
      ma.b2 = bias_k[2];
      ma.wout = wout_k;
      ma.bout = bout_k;
      ma.erow = erow_k;
      ma.D1 = reinterpret_cast<bf16_t*>(D1k);
      ma.ld_d1 = ldd1;
      ma.escale = escale;
      if (io.dparams) {
        ma.H2 = reinterpret_cast<bf16_t*>(H2);
        ma.H3 = reinterpret_cast<bf16_t*>(H3);
        ma.D3 = reinterpret_cast<bf16_t*>(D3);
        ma.D2 = reinterpret_cast<bf16_t*>(D2);
        ma.uprow = at<float>(ws, P.uprow);
      }
      ma.perm = perm;
      ma.mol = mol;
      ma.dLdE = io.dLdE;
      ma.alpha = h->alpha;
      ma.inv_alpha_l2e = g.inv_alpha_l2e;
      StageTimer t(h, io.timed, ST_MID, st);
      fused = launch_mlp_mid(h->width, ma, P.rows_cap, st);
    }
    if (!fused) {
      // layer 2: H2 = CELU(H1 W1^T + b1)
      g.A = H1; g.lda = w1; g.B = Wk[1]; g.Bq = Wqk[1]; g.sB = (long)w2 * w1; g.ldb = w1;
      g.bias = bias_k[1]; g.sBias = w2; g.N = w2; g.K = w1; g.C = H2; g.ldc = w2;
      {
        StageTimer t(h, io.timed, ST_L2, st);
        ok &= launch_gemm<T>(EPI_CELU, g, P.rows_cap, st);
      }
      // layer 3 + output: E_i, delta3
      g.A = H2; g.lda = w2; g.B = Wk[2]; g.Bq = nullptr; g.sB = (long)w3 * w2; g.ldb = w2;
      g.bias = bias_k[2]; g.sBias = w3; g.N = w3; g.K = w2;
      g.C = need_bwd ? (void*)D3 : nullptr; g.ldc = w3;
      g.w_out = wout_k; g.sWout = w3; g.b_out = bout_k; g.erow = erow_k;
      g.H3 = io.dparams ? (void*)H3 : nullptr; g.ldh3 = w3;
      g.perm = perm; g.mol = mol; g.dLdE = io.dLdE;
      g.uprow = io.dparams ? at<float>(ws, P.uprow) : nullptr;
      {
        StageTimer t(h, io.timed, ST_HEAD, st);
        ok &= launch_gemm<T>(EPI_HEAD, g, P.rows_cap, st);
      }
      g.H3 = nullptr;
      g.uprow = nullptr;
      if (need_bwd) {
        // delta2 = (delta3 W2) * CELU'(z2)
        g.A = D3; g.lda = w3; g.B = WTk[2]; g.Bq = WTqk[2]; g.sB = (long)w2 * w3; g.ldb = w3;
        g.bias = nullptr; g.N = w2; g.K = w3; g.C = D2; g.ldc = w2; g.H = H2; g.ldh = w2;
        {
          StageTimer t(h, io.timed, ST_BWD3, st);
          ok &= launch_gemm<T>(EPI_BWD, g, P.rows_cap, st);
        }
        // delta1 = (delta2 W1) * CELU'(z1)
        g.A = D2; g.lda = w2; g.B = WTk[1]; g.Bq = WTqk[1]; g.sB = (long)w1 * w2; g.ldb = w2;
        g.N = w1; g.K = w2; g.C = D1k; g.ldc = ldd1; g.H = H1; g.ldh = w1;
        {
          StageTimer t(h, io.timed, ST_BWD2, st);
          ok &= launch_gemm<T>(EPI_BWD, g, P.rows_cap, st);
        }
      }
    }
  }  // members
  // the molecular energies: beside the force scatter when there is one
  const EnergyArgs ea{io.off, xyzs, erow, M, (long)P.rows_cap, h->eself, io.E, status};
  if (io.E && !io.out3) {
    StageTimer t(h, io.timed, ST_ENERGY, st);
    launch_energy(dims, P.nmol, io.off, xyzs, erow, M, (long)P.rows_cap, h->eself, io.E, status,
                  st);
  }
  if (io.out3) {
    // g = dE/dG = delta1 W0 (in the network operand type)
    // (ensembles: one product over the members' delta1 side by side and the
    // member-concatenated W0^T, so the mean of their dE/dG is accumulated in
    // FP32 inside the product; the 1/M is already in delta1)
    GemmArgs g{};
    g.gt = gt;
    g.alpha = h->alpha;
    g.inv_alpha_l2e = (float)(1.4426950408889634 / h->alpha);
    const bool cat = M > 1;
    g.A = D1; g.lda = ldd1;
    g.B = cat ? (bf ? nullptr : (const void*)h->WT0cf) : WT[0];
    g.Bq = cat ? (bf ? (const void*)h->WT0cq : nullptr) : WTq[0];
    g.sB = (long)Fp * ldd1; g.ldb = ldd1;
    g.N = Fp; g.K = ldd1; g.C = G; g.ldc = Fp; g.H = nullptr;
    g.kmask_n = kmask;  // the adjoint reads a row's own k-steps of dE/dG only
    if (!net_fused) {
      StageTimer t(h, io.timed, ST_GRADG, st);
      ok &= launch_gemm<T>(EPI_OUT, g, P.rows_cap, st);
    }
    StageTimer t(h, io.timed, ST_AEVBWD, st);
    float4* pgrad = h->deterministic ? at<float4>(ws, P.pgrad) : nullptr;
    launch_aev_bwd<T>(dims, P.n, h->C, rec, nbr, counts, P.cap, row, G, Fp, io.out3, io.sign,
                      io.gidx, io.n_total, mrange, &ea, P.nmol, pgrad, st);
    if (pgrad)
      launch_force_gather(dims, P.n, xyzs, rec, nbr, counts, P.cap, pgrad, io.out3, io.sign,
                          io.gidx, io.n_total, st);
  }
  if (io.dparams) {
    StageTimer t(h, io.timed, ST_WGRAD, st);
    float* part = at<float>(ws, P.wpart);
    const float* up = at<float>(ws, P.uprow);
    const WgradLayer layers[kLayers] = {
        {D1, X, w1, Fp, w1, h->F, false, S * kNR, h->C.A0 - S * kNR},
        {D2, H1, w2, w1, w2, w1, false},
        {D3, H2, w3, w2, w3, w2, false},
        {up, H3, 1, w3, 1, w3, true},
    };
    launch_wgrad_net<T>(gt, S, P.nwchunks, kWChunk, layers, kLayers, part, io.dparams,
                        h->param_off_dev, st);
  }
  if (!ok) return NNP_E_INVALID;
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

nnp_status run(nnp_handle* h, const Plan& P, void* ws, const EvalIO& io, hipStream_t st) {
  if (h->prec == NNP_MLP_BF16) return run_path<bf16_t>(h, P, ws, io, st);
  return run_path<float>(h, P, ws, io, st);
}

// groups: with a box, mol_offsets may split the atoms into energy groups
// (all atoms still interact); only the owned/ghost entry point does that.
nnp_status check_common(nnp_handle* h, int n, int nmol, const float* pos, const int* species,
                        const int* off, const float* box, void* ws, size_t ws_bytes, Plan& P,
                        bool groups = false) {
  if (!h || n < 0 || nmol < 1) return NNP_E_INVALID;
  if (n > 0 && (!pos || !species)) return NNP_E_INVALID;
  if (!off) return NNP_E_INVALID;
  if (n >= (1 << 27)) return NNP_E_INVALID;
  if (box && nmol != 1 && !groups) return NNP_E_INVALID;
  BoxConst B;
  if (!make_box(h, box, B)) return NNP_E_BOX;
  P = make_plan(h, n, nmol, B);
  if (!ws || ws_bytes < P.total) return NNP_E_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return NNP_E_HIP;
  return NNP_OK;
}

}  // namespace

// =================================================================== C ABI

extern "C" {

const char* nnp_status_string(nnp_status s) {
  switch (s) {
    case NNP_OK: return "ok";
    case NNP_E_INVALID: return "invalid argument";
    case NNP_E_SPECIES: return "species index out of range";
    case NNP_E_BOX: return "box edge shorter than twice the radial cutoff";
    case NNP_E_CAPACITY: return "neighbor list capacity exceeded";
    case NNP_E_OOM: return "device out of memory";
    case NNP_E_HIP: return "HIP runtime error";
    case NNP_E_NONFINITE: return "non-finite position or energy";
    case NNP_E_WORKSPACE: return "workspace missing or too small";
    case NNP_E_BUSY: return "server has no capacity for the request";
  }
  return "unknown status";
}

nnp_status nnp_create(const nnp_aev_params* aev, const nnp_mlp_params* mlp,
                      nnp_precision precision, nnp_handle** out) {
  return nnp_create_ensemble(aev, mlp, 1, precision, out);
}

nnp_status nnp_create_ensemble(const nnp_aev_params* aev, const nnp_mlp_params* mlps,
                               int32_t n_models, nnp_precision precision, nnp_handle** out) {
  if (!aev || !mlps || !out) return NNP_E_INVALID;
  *out = nullptr;
  if (n_models < 1 || n_models > kMaxModels) return NNP_E_INVALID;
  const nnp_mlp_params* mlp = &mlps[0];
  const int S = aev->n_species;
  if (S < 1 || S > kMaxS) return NNP_E_INVALID;
  if (aev->n_shf_r != kNR || aev->n_shf_a != kNA || aev->n_shf_z != kNZ) return NNP_E_INVALID;
  if (!aev->shf_r || !aev->shf_a || !aev->shf_z) return NNP_E_INVALID;
  if (!(aev->rc_rad > 0.f) || !(aev->rc_ang > 0.f) || aev->rc_ang > aev->rc_rad)
    return NNP_E_INVALID;
  if (!(aev->angle_cos_scale > 0.f && aev->angle_cos_scale < 1.f)) return NNP_E_INVALID;
  if (precision != NNP_MLP_FP32 && precision != NNP_MLP_BF16) return NNP_E_INVALID;
  if (mlp->n_layers != kLayers || !mlp->width || !mlp->params) return NNP_E_INVALID;
  const int F = kNR * S + 32 * S * (S + 1) / 2;
  if (mlp->width[0] != F || mlp->width[kLayers] != 1) return NNP_E_INVALID;
  for (int l = 1; l < kLayers; ++l)
    if (mlp->width[l] < 32 || mlp->width[l] > 256 || mlp->width[l] % 32) return NNP_E_INVALID;
  if (!(mlp->celu_alpha > 0.f)) return NNP_E_INVALID;
  for (int k = 1; k < n_models; ++k) {  // members share the architecture
    const nnp_mlp_params& q = mlps[k];
    if (q.n_layers != kLayers || !q.width || !q.params || q.celu_alpha != mlp->celu_alpha)
      return NNP_E_INVALID;
    for (int l = 0; l <= kLayers; ++l)
      if (q.width[l] != mlp->width[l]) return NNP_E_INVALID;
  }

  nnp_handle* h = new (std::nothrow) nnp_handle();
  if (!h) return NNP_E_OOM;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return NNP_E_HIP;
  }
  // the allocation-free entry point's scratch address on this device (a
  // failed lookup is retried, and reported, by that entry point)
  (void)scratch_ptr(h->device);
  h->prec = precision;
  h->S = S;
  h->F = F;
  const int A0 = (S * kNR + 31) / 32 * 32;  // the angular blocks on k-step boundaries
  h->Fp = (A0 + (F - S * kNR) + 63) / 64 * 64;
  for (int l = 0; l <= kLayers; ++l) h->width[l] = mlp->width[l];
  h->alpha = mlp->celu_alpha;
  AevConst& C = h->C;
  C.S = S;
  C.F = F;
  C.Fp = h->Fp;
  C.A0 = A0;
  const float rr = aev->rc_rad, ra = aev->rc_ang;
  C.rc2_r = rr * rr;
  C.rc2_a = ra * ra;
  C.inv_rc_r = 1.0f / rr;
  C.inv_rc_a = 1.0f / ra;
  C.pi_2rc_r = (float)(M_PI / (2.0 * rr));
  C.pi_2rc_a = (float)(M_PI / (2.0 * ra));
  const double l2e = 1.4426950408889634;
  C.eta_r_l2e = (float)(aev->eta_r * l2e);
  C.eta_r2 = 2.f * aev->eta_r;
  C.eta_a_l2e = (float)(aev->eta_a * l2e);
  C.eta_a = aev->eta_a;
  C.zeta = aev->zeta;
  C.cR = aev->radial_prefactor;
  C.kappa = aev->angle_cos_scale;
  for (int m = 0; m < kNR; ++m) C.shf_r[m] = aev->shf_r[m];
  for (int a = 0; a < kNA; ++a) C.shf_a[a] = aev->shf_a[a];
  for (int z = 0; z < kNZ; ++z) {
    C.cos_z[z] = (float)std::cos((double)aev->shf_z[z]);
    C.sin_z[z] = (float)std::sin((double)aev->shf_z[z]);
  }
  // flat parameter offsets: member-major, then element, then layer
  h->n_models = n_models;
  const int Q = n_models * S;  // weight slots
  size_t o = 0;
  for (int q = 0; q < Q; ++q)
    for (int l = 0; l < kLayers; ++l) {
      h->param_off[q][l] = (long)o;
      o += (size_t)h->width[l + 1] * h->width[l] + h->width[l + 1];
    }
  h->n_params = o;
  const size_t per_model = o / n_models;
  // one device allocation for all weight copies
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t a = bytes;
    bytes = align_up(bytes + b, 256);
    return a;
  };
  const size_t o_flat = take(o * 4);
  size_t o_wf[kLayers], o_wb[kLayers], o_wtf[kLayers], o_wqb[kLayers], o_wtqb[kLayers],
      o_b[kLayers];
  for (int l = 0; l < kLayers - 1; ++l) {
    const size_t inp = l == 0 ? h->Fp : h->width[l];
    const size_t el = (size_t)Q * h->width[l + 1] * inp;
    o_wf[l] = take(el * 4);
    o_wb[l] = take(el * 2);
    o_wtf[l] = take(el * 4);
    o_wqb[l] = take(el * 2);
    o_wtqb[l] = take(el * 2);
    o_b[l] = take((size_t)Q * h->width[l + 1] * 4);
  }
  const size_t cat_el = n_models > 1 ? (size_t)S * h->Fp * n_models * h->width[1] : 0;
  const size_t o_wt0cf = take(cat_el * 4);
  const size_t o_wt0cq = take(cat_el * 2);
  const size_t o_wout = take((size_t)Q * h->width[3] * 4);
  const size_t o_bout = take((size_t)Q * 4);
  const size_t o_eself = take(kMaxS * 8);
  const size_t o_poff = take((size_t)kLayers * S * 8);
  const size_t o_lane = take((size_t)(kNR + 2 * kNZ) * 4);
  if (hipMalloc(&h->dmem, bytes) != hipSuccess) {
    delete h;
    return NNP_E_OOM;
  }
  h->flat = reinterpret_cast<float*>(h->dmem + o_flat);
  for (int l = 0; l < kLayers - 1; ++l) {
    h->Wf[l] = reinterpret_cast<float*>(h->dmem + o_wf[l]);
    h->Wb[l] = reinterpret_cast<bf16_t*>(h->dmem + o_wb[l]);
    h->WTf[l] = reinterpret_cast<float*>(h->dmem + o_wtf[l]);
    h->Wqb[l] = reinterpret_cast<bf16_t*>(h->dmem + o_wqb[l]);
    h->WTqb[l] = reinterpret_cast<bf16_t*>(h->dmem + o_wtqb[l]);
    h->bias[l] = reinterpret_cast<float*>(h->dmem + o_b[l]);
  }
  if (n_models > 1) {
    h->WT0cf = reinterpret_cast<float*>(h->dmem + o_wt0cf);
    h->WT0cq = reinterpret_cast<bf16_t*>(h->dmem + o_wt0cq);
  }
  h->wout = reinterpret_cast<float*>(h->dmem + o_wout);
  h->bout = reinterpret_cast<float*>(h->dmem + o_bout);
  h->eself = reinterpret_cast<double*>(h->dmem + o_eself);
  h->param_off_dev = reinterpret_cast<long*>(h->dmem + o_poff);
  C.lane_tab = reinterpret_cast<const float*>(h->dmem + o_lane);
  float lane_host[kNR + 2 * kNZ];
  for (int m = 0; m < kNR; ++m) lane_host[m] = C.shf_r[m];
  for (int z = 0; z < kNZ; ++z) {
    lane_host[kNR + z] = C.cos_z[z];
    lane_host[kNR + kNZ + z] = C.sin_z[z];
  }

  double es[kMaxS] = {};
  for (int s = 0; s < S; ++s) es[s] = mlp->self_energy ? mlp->self_energy[s] : 0.0;
  std::vector<long> po((size_t)kLayers * S);
  for (int l = 0; l < kLayers; ++l)
    for (int s = 0; s < S; ++s) po[(size_t)l * S + s] = h->param_off[s][l];
  bool ok = true;
  for (int k = 0; k < n_models && ok; ++k)
    ok = hip_ok(hipMemcpy(h->flat + k * per_model, mlps[k].params, per_model * 4,
                          hipMemcpyHostToDevice));
  ok = ok && hip_ok(hipMemcpy(h->eself, es, sizeof(es), hipMemcpyHostToDevice)) &&
            hip_ok(hipMemcpy(h->param_off_dev, po.data(), po.size() * 8, hipMemcpyHostToDevice)) &&
            hip_ok(hipMemcpy(const_cast<float*>(C.lane_tab), lane_host, sizeof(lane_host),
                             hipMemcpyHostToDevice));
  if (ok) ok = nnp_set_params_device(h, h->flat, nullptr) == NNP_OK &&
               hip_ok(hipDeviceSynchronize());
  if (!ok) {
    (void)hipFree(h->dmem);
    delete h;
    return NNP_E_HIP;
  }
  *out = h;
  return NNP_OK;
}

void nnp_destroy(nnp_handle* h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  for (hipEvent_t ev : h->ev_pool) (void)hipEventDestroy(ev);
  if (h->dmem) (void)hipFree(h->dmem);
  delete h;
}

size_t nnp_param_count(const nnp_handle* h) { return h ? h->n_params : 0; }

nnp_status nnp_set_params_device(nnp_handle* h, const float* params_dev, void* stream) {
  if (!h || !params_dev) return NNP_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (params_dev != h->flat &&
      hipMemcpyAsync(h->flat, params_dev, h->n_params * 4, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return NNP_E_HIP;
  PackArgs p{};
  p.flat = h->flat;
  const int Q = h->n_models * h->S;
  for (int q = 0; q < Q; ++q)
    for (int l = 0; l < kLayers; ++l) p.off[q * kLayers + l] = h->param_off[q][l];
  p.S = h->S;
  p.n_models = h->n_models;
  p.WT0cf = h->WT0cf;
  p.WT0cq = h->WT0cq;
  for (int l = 0; l <= kLayers; ++l) p.width[l] = h->width[l];
  p.width[0] = h->F;
  p.Fp = h->Fp;
  p.r0 = h->S * kNR;
  p.a0 = h->C.A0;
  for (int l = 0; l < kLayers; ++l) {
    p.Wf[l] = h->Wf[l];
    p.Wb[l] = h->Wb[l];
    p.WTf[l] = h->WTf[l];
    p.Wqb[l] = h->Wqb[l];
    p.WTqb[l] = h->WTqb[l];
    p.bias[l] = h->bias[l];
  }
  p.wout = h->wout;
  p.bout = h->bout;
  launch_pack(p, Q, st);
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

nnp_status nnp_profile_enable(nnp_handle* h, int on) {
  if (!h) return NNP_E_INVALID;
  h->prof = on != 0;
  h->ev_pending.clear();
  h->ev_next = 0;
  for (int i = 0; i < 32; ++i) {
    h->prof_ms[i] = 0.0;
    h->prof_n[i] = 0;
  }
  return NNP_OK;
}

nnp_status nnp_profile_collect(nnp_handle* h, void* stream) {
  if (!h) return NNP_E_INVALID;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return NNP_E_HIP;
  for (auto& p : h->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) != hipSuccess) return NNP_E_HIP;
    h->prof_ms[p.first] += ms;
    h->prof_n[p.first] += 1;
  }
  h->ev_pending.clear();
  h->ev_next = 0;
  return NNP_OK;
}

int32_t nnp_profile_stage_count(void) { return ST_COUNT; }

const char* nnp_profile_stage_name(int32_t i) {
  return (i >= 0 && i < ST_COUNT) ? kStageNames[i] : "";
}

nnp_status nnp_profile_read(const nnp_handle* h, double* total_ms, int64_t* count, int32_t max) {
  if (!h) return NNP_E_INVALID;
  for (int i = 0; i < max && i < ST_COUNT; ++i) {
    if (total_ms) total_ms[i] = h->prof_ms[i];
    if (count) count[i] = h->prof_n[i];
  }
  return NNP_OK;
}

nnp_status nnp_set_triclinic(nnp_handle* h, int32_t on) {
  if (!h) return NNP_E_INVALID;
  h->triclinic = on != 0;
  return NNP_OK;
}

nnp_status nnp_set_deterministic(nnp_handle* h, int32_t on) {
  if (!h) return NNP_E_INVALID;
  h->deterministic = on != 0;
  return NNP_OK;
}

nnp_status nnp_set_max_neighbors(nnp_handle* h, int32_t m) {
  if (!h || m < 16 || m > 512) return NNP_E_INVALID;
  h->max_nbr = (m + 15) / 16 * 16;  // keeps the per-wave LDS regions 16-byte aligned
  return NNP_OK;
}

size_t nnp_workspace_bytes(const nnp_handle* h, int32_t n, int32_t nmol, const float* box) {
  if (!h || n < 0 || nmol < 1) return 0;
  BoxConst B;
  if (!make_box(h, box, B)) return 0;
  return make_plan(h, n, nmol, B).total;
}

nnp_status nnp_energy_forces(nnp_handle* h, int32_t n, int32_t nmol, const float* pos,
                             const int32_t* species, const int32_t* off, const float* box,
                             double* E, float* F, void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  nnp_status s = check_common(h, n, nmol, pos, species, off, box, ws, ws_bytes, P);
  if (s != NNP_OK) return s;
  if (!E) return NNP_E_INVALID;
  EvalIO io{n, nmol, pos, nullptr, species, off, E, F, 1.f, nullptr, nullptr};
  return run(h, P, ws, io, static_cast<hipStream_t>(stream));
}

nnp_status nnp_energy_forces_noalloc(nnp_handle* h, int32_t n, int32_t nmol, const float* pos,
                                     const int32_t* species, const int32_t* off,
                                     const float* box, double* E, float* F, uint32_t* status,
                                     void* stream) {
  if (!h || n < 0 || nmol < 1 || !E) return NNP_E_INVALID;
  if (n > 0 && (!pos || !species)) return NNP_E_INVALID;
  if (!off || (box && nmol != 1) || n >= (1 << 27)) return NNP_E_INVALID;
  BoxConst B;
  if (!make_box(h, box, B)) return NNP_E_BOX;
  const Plan P = make_plan(h, n, nmol, B, false);
  if (P.total > kScratchBytes) return NNP_E_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return NNP_E_HIP;
  void* ws = scratch_ptr(h->device);
  if (!ws) return NNP_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  EvalIO io{n, nmol, pos, nullptr, species, off, E, F, 1.f, nullptr, nullptr};
  io.timed = false;  // stage events would create HIP events
  const nnp_status s = run(h, P, ws, io, st);
  if (s != NNP_OK) return s;
  if (status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st,
                       static_cast<const uint32_t*>(at<uint32_t>(ws, P.status)), status);
    if (!launches_ok()) return NNP_E_HIP;
  }
  return NNP_OK;
}

nnp_status nnp_energy_forces_subset(nnp_handle* h, int32_t n_sub, int32_t nmol,
                                    const int32_t* idx, int32_t n_total, const float* pos_all,
                                    const int32_t* species, const int32_t* off,
                                    const float* box, double* E, float* F_all, void* ws,
                                    size_t ws_bytes, void* stream) {
  if (!idx || n_total < 1 || !pos_all) return NNP_E_INVALID;
  Plan P;
  nnp_status s = check_common(h, n_sub, nmol, pos_all, species, off, box, ws, ws_bytes, P);
  if (s != NNP_OK) return s;
  if (!E) return NNP_E_INVALID;
  EvalIO io{n_sub, nmol, pos_all, nullptr, species, off, E, F_all, 1.f, nullptr, nullptr};
  io.gidx = idx;
  io.n_total = n_total;
  return run(h, P, ws, io, static_cast<hipStream_t>(stream));
}

nnp_status nnp_backward(nnp_handle* h, int32_t n, int32_t nmol, const float* pos,
                        const int32_t* species, const int32_t* off, const float* box,
                        const double* dLdE, float* dL_dpos, float* dL_dparams, double* E,
                        void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  nnp_status s = check_common(h, n, nmol, pos, species, off, box, ws, ws_bytes, P);
  if (s != NNP_OK) return s;
  if (!dLdE) return NNP_E_INVALID;
  if (dL_dparams && h && h->n_models > 1) return NNP_E_INVALID;  // weight gradients: one network
  EvalIO io{n, nmol, pos, nullptr, species, off, E, dL_dpos, -1.f, dLdE, dL_dparams};
  return run(h, P, ws, io, static_cast<hipStream_t>(stream));
}

nnp_status nnp_energy_forces_owned(nnp_handle* h, int32_t n, int32_t n_owned, const float* pos,
                                   const int32_t* species, const float* box, double* E, float* F,
                                   void* ws, size_t ws_bytes, void* stream) {
  if (!h || n < 1 || n_owned < 0 || n_owned > n || !box || !E || !F || !ws) return NNP_E_INVALID;
  // the group arrays live in the workspace: plan once to find them, then
  // check everything with them in place
  BoxConst B;
  if (!make_box(h, box, B)) return NNP_E_BOX;
  const Plan P0 = make_plan(h, n, 2, B);
  if (ws_bytes < P0.total) return NNP_E_WORKSPACE;
  int* off = at<int>(ws, P0.grp);
  double* up = reinterpret_cast<double*>(static_cast<char*>(ws) + P0.grp + 16);
  Plan P;
  nnp_status s = check_common(h, n, 2, pos, species, off, box, ws, ws_bytes, P, true);
  if (s != NNP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_owned_groups, dim3(1), dim3(64), 0, st, n, n_owned, off, up);
  // forces of the owned energy: the adjoint with upstream 1 for group 0 and 0
  // for the ghosts, written as forces (sign +1)
  EvalIO io{n, 2, pos, nullptr, species, off, E, F, 1.f, up, nullptr};
  return run(h, P, ws, io, st);
}

nnp_status nnp_check(const nnp_handle* h, void* ws, void* stream) {
  if (!h || !ws) return NNP_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return NNP_E_HIP;
  uint32_t word = 0;
  if (hipMemcpy(&word, ws, 4, hipMemcpyDeviceToHost) != hipSuccess) return NNP_E_HIP;
  if (word & kStOffsets) return NNP_E_INVALID;
  if (word & kStSpecies) return NNP_E_SPECIES;
  if (word & kStNonFinite) return NNP_E_NONFINITE;
  if (word & kStCapacity) return NNP_E_CAPACITY;
  return NNP_OK;
}

nnp_status nnp_debug_neighbors(nnp_handle* h, int32_t n, void* ws, size_t ws_bytes,
                               int32_t* counts, int32_t* nbr, void* stream) {
  if (!h || !ws || n < 0) return NNP_E_INVALID;
  BoxConst B;
  make_box(h, nullptr, B);
  // the neighbor and count arrays sit at the same offsets with and without a box
  Plan P = make_plan(h, n, 1, B);
  if (ws_bytes < P.total) return NNP_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (counts && hipMemcpyAsync(counts, at<char>(ws, P.counts), (size_t)n * 8,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
    return NNP_E_HIP;
  if (nbr && hipMemcpyAsync(nbr, at<char>(ws, P.nbr), (size_t)n * P.cap * 4,
                            hipMemcpyDeviceToDevice, st) != hipSuccess)
    return NNP_E_HIP;
  return NNP_OK;
}

nnp_status nnp_debug_atom_energies(nnp_handle* h, int32_t n, int32_t nmol, const float* box,
                                   void* ws, size_t ws_bytes, float* e_atom, void* stream) {
  if (!h || !ws || !e_atom || n < 0 || nmol < 1) return NNP_E_INVALID;
  BoxConst B;
  if (!make_box(h, box, B)) return NNP_E_BOX;
  const Plan P = make_plan(h, n, nmol, B);
  if (ws_bytes < P.total) return NNP_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int k = 0; k < h->n_models; ++k)
    if (hipMemcpyAsync(e_atom + (size_t)k * n, at<float>(ws, P.erow) + (size_t)k * P.rows_cap,
                       (size_t)n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return NNP_E_HIP;
  return NNP_OK;
}

nnp_status nnp_debug_aev(nnp_handle* h, int32_t n, int32_t nmol, const float* pos,
                         const int32_t* species, const int32_t* off, const float* box, float* aev,
                         void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  nnp_status s = check_common(h, n, nmol, pos, species, off, box, ws, ws_bytes, P);
  if (s != NNP_OK) return s;
  if (!aev) return NNP_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* dims = at<int>(ws, P.dims);
  uint32_t* status = at<uint32_t>(ws, P.status);
  float4* xyzs = at<float4>(ws, P.xyzs);
  int2* mrange = P.mrange ? at<int2>(ws, P.mrange) : nullptr;
  launch_stage(n, nmol, P.n, dims, pos, nullptr, nullptr, 0, species, off, h->S, xyzs,
               at<int>(ws, P.mol), mrange, nullptr, at<int>(ws, P.hist), status, true,
               P.B.periodic ? at<int>(ws, P.cell_cnt) : nullptr, P.B.periodic ? cell_zero_ints(P.ncell) : 0,
               st);
  launch_groups(dims, P.n, h->S, at<int>(ws, P.hist), at<GroupTable>(ws, P.gt),
                at<int>(ws, P.perm), P.rows_cap, off, kWChunk, status, st);
  if (P.B.periodic)
    launch_pairs_cell(dims, P.n, h->C, P.B, xyzs, at<int>(ws, P.cell_of), at<int>(ws, P.cell_cnt),
                      at<int>(ws, P.cell_start), at<int>(ws, P.cursor), at<int>(ws, P.cell_atoms),
                      at<float4>(ws, P.cell_xyzs), P.cap, at<int>(ws, P.nbr),
                      at<float4>(ws, P.rec), at<int2>(ws, P.counts), status, st);
  else
    launch_pairs_mol(dims, P.n, h->C, xyzs, mrange, P.cap, at<int>(ws, P.nbr),
                     at<float4>(ws, P.rec), at<int2>(ws, P.counts), status, st);
  AevConst Cp = h->C;  // rows in the published order: no gap before the angular blocks
  Cp.A0 = h->S * kNR;
  launch_aev_fwd<float>(dims, P.n, Cp, at<float4>(ws, P.rec), at<int2>(ws, P.counts), P.cap,
                        nullptr, aev, h->F, h->deterministic, nullptr, false, st);
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

// ------------------------------------------------------------- graph replay

}  // extern "C"

struct nnp_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

extern "C" {

nnp_status nnp_graph_capture(nnp_handle* h, int32_t n, int32_t nmol, const float* pos,
                             const int32_t* species, const int32_t* off, const float* box,
                             double* E, float* F, void* ws, size_t ws_bytes, void* stream,
                             nnp_graph** out) {
  if (!out || !stream) return NNP_E_INVALID;
  *out = nullptr;
  if (h && h->prof) return NNP_E_INVALID;  // event timing cannot be captured
  // eager run: validates the arguments and sets kernel attributes
  nnp_status s = nnp_energy_forces(h, n, nmol, pos, species, off, box, E, F, ws, ws_bytes, stream);
  if (s != NNP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return NNP_E_HIP;
  s = nnp_energy_forces(h, n, nmol, pos, species, off, box, E, F, ws, ws_bytes, stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(st, &g);
  if (s != NNP_OK || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return s != NNP_OK ? s : NNP_E_HIP;
  }
  nnp_graph* G = new (std::nothrow) nnp_graph();
  if (!G) {
    (void)hipGraphDestroy(g);
    return NNP_E_OOM;
  }
  G->graph = g;
  G->device = h->device;
  if (hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    delete G;
    return NNP_E_HIP;
  }
  *out = G;
  return NNP_OK;
}

nnp_status nnp_graph_launch(nnp_graph* g, void* stream) {
  if (!g || !g->exec) return NNP_E_INVALID;
  return hip_ok(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream))) ? NNP_OK : NNP_E_HIP;
}

void nnp_graph_destroy(nnp_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ------------------------------------------------------------------------- MD

nnp_status nnp_md_steps(nnp_handle* h, int32_t n, int32_t nmol, double* x, double* v, float* F,
                        const double* mass, const int32_t* species, const int32_t* off,
                        const float* box, double dt, int32_t n_steps, double* E_pot,
                        double* E_kin, void* ws, size_t ws_bytes, void* stream) {
  if (!x || !v || !F || !mass || n_steps < 0 || !(dt > 0.0)) return NNP_E_INVALID;
  Plan P;
  float* pos32 = nullptr;
  {
    // positions are staged inside the workspace: validate with a dummy non-null pointer
    nnp_status s = check_common(h, n, nmol, reinterpret_cast<const float*>(x), species, off, box,
                                ws, ws_bytes, P);
    if (s != NNP_OK) return s;
    pos32 = at<float>(ws, P.pos32);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* dims = at<int>(ws, P.dims);
  // dims are written by the first force evaluation; integration kernels read them
  double* Etmp = E_pot;
  std::vector<double> dummy;
  nnp_status s = NNP_OK;
  for (int k = 0; k < n_steps && s == NNP_OK; ++k) {
    if (k == 0) {
      // the staging kernel of the first evaluation has not run yet: use counts by value
      launch_fill_i32(dims, n, 1, st);
      launch_fill_i32(dims + 1, nmol, 1, st);
    }
    launch_vv_kick_drift(dims, n, x, v, F, mass, dt, pos32, st);
    EvalIO io{n, nmol, pos32, nullptr, species, off, Etmp, F, 1.f, nullptr, nullptr};
    io.keep_status = k > 0;  // the segment's device errors accumulate
    s = run(h, P, ws, io, st);
    if (s != NNP_OK) break;
    launch_vv_kick(dims, n, v, F, mass, dt, st);
  }
  if (s == NNP_OK && E_kin) {
    if (n_steps == 0) {
      launch_fill_i32(dims, n, 1, st);
      launch_fill_i32(dims + 1, nmol, 1, st);
    }
    launch_kinetic(dims, nmol, off, v, mass, E_kin, nullptr, st);
  }
  if (s != NNP_OK) return s;
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

nnp_status nnp_langevin_steps(nnp_handle* h, int32_t n, int32_t nmol, double* x, double* v,
                              float* F, const double* mass, const int32_t* species,
                              const int32_t* off, const float* box, double dt, int32_t n_steps,
                              double temperature, double friction, uint64_t seed, uint64_t step0,
                              double* E_pot, double* E_kin, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!x || !v || !F || !mass || n_steps < 0 || !(dt > 0.0) || !(temperature >= 0.0) ||
      !(friction >= 0.0))
    return NNP_E_INVALID;
  Plan P;
  float* pos32 = nullptr;
  {
    nnp_status s = check_common(h, n, nmol, reinterpret_cast<const float*>(x), species, off, box,
                                ws, ws_bytes, P);
    if (s != NNP_OK) return s;
    pos32 = at<float>(ws, P.pos32);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  int* dims = at<int>(ws, P.dims);
  const double kB = 8.617333262e-5;         // eV / K
  const double acc = 9.648533e-3;           // A/fs^2 per eV/A/amu
  const double c = std::exp(-friction * 1e-3 * dt);  // friction in 1/ps, dt in fs
  const double kT_acc = kB * temperature * acc;
  nnp_status s = NNP_OK;
  // the integration kernel reads the atom count the staging kernel writes;
  // before the first evaluation of this call it is set here
  launch_fill_i32(dims, n, 1, st);
  launch_fill_i32(dims + 1, nmol, 1, st);
  for (int k = 0; k < n_steps && s == NNP_OK; ++k) {
    launch_lfm_step(dims, n, x, v, F, mass, dt, c, kT_acc, seed, step0 + (uint64_t)k, pos32, st);
    EvalIO io{n, nmol, pos32, nullptr, species, off, E_pot, F, 1.f, nullptr, nullptr};
    s = run(h, P, ws, io, st);
  }
  if (s == NNP_OK && E_kin) launch_kinetic(dims, nmol, off, v, mass, E_kin, nullptr, st);
  if (s != NNP_OK) return s;
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

}  // extern "C"

// =================================================================== serving

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  int64_t id = 0;
  int n = 0;
  int n_steps = 0;
  int k = 0;  // steps issued (host mirror of the device counter)
  std::vector<double> x, v;
  std::vector<int> sp;
  double t_submit = 0, t_admit = 0, t_done = 0;
  double e_pot = 0, e_kin = 0;
  uint32_t status = 0;  // device status bits seen while the request was on the device
};

// Results of the requests that finished in one round, on their way to the
// host: device-to-host copies into a pinned buffer behind an event, read on a
// later round (or when the server runs dry), so no round waits for the GPU.
struct RetireSlot {
  hipEvent_t ev = nullptr;
  double* h = nullptr;  // x, v per request, then the batch's E_pot, E_kin, then the status word
  std::vector<std::pair<Req*, size_t>> reqs;  // finishing request, offset of its x in h
  std::vector<int> mol;                       // its molecule index in the batch
  std::vector<Req*> exposed;  // requests on the device while the status bits accumulated
  size_t eo = 0;              // offset of the energies in h
  int nact = 0;               // molecules in the batch
};
constexpr int kRetireSlots = 4;

}  // namespace

struct nnp_server {
  nnp_handle* h = nullptr;
  int device = 0;  // the handle's device, kept so destruction never reads the handle
  hipStream_t st = nullptr;
  double dt = 0.5;
  // integrator: velocity Verlet, or LF-Middle Langevin after nnp_server_set_langevin
  bool lfm = false;
  double lfm_c = 1.0, lfm_kT = 0.0;
  double mass_tab[kMaxS] = {};
  int max_atoms = 0, max_mols = 0;
  size_t bytes = 0;
  char* dmem = nullptr;
  // active state (fixed addresses: the step graph refers to them)
  double *x = nullptr, *v = nullptr, *m = nullptr;
  int* sp = nullptr;
  float* F = nullptr;
  float* pos32 = nullptr;
  int *off = nullptr, *kdone = nullptr, *nsteps = nullptr;
  double *epot = nullptr, *ekin = nullptr;
  uint64_t* seed = nullptr;  // per molecule: the request id (Langevin noise key)
  // repack scratch and staging of admitted atoms
  double *x2 = nullptr, *v2 = nullptr, *m2 = nullptr;
  int* sp2 = nullptr;
  float* F2 = nullptr;
  int* src = nullptr;
  double *in_x = nullptr, *in_v = nullptr, *in_m = nullptr;
  int* in_sp = nullptr;
  void* ws = nullptr;
  Plan P;
  // pinned host mirrors
  char* hmem = nullptr;
  int *h_src = nullptr, *h_off = nullptr, *h_kdone = nullptr, *h_nsteps = nullptr,
      *h_dims = nullptr, *h_in_sp = nullptr;
  double *h_in_x = nullptr, *h_in_v = nullptr, *h_in_m = nullptr, *h_out = nullptr;
  uint64_t* h_seed = nullptr;
  hipEvent_t ev_upload = nullptr;
  // graph of one step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool warmed = false;
  // requests
  std::deque<Req*> pending;
  std::vector<Req*> active;
  std::map<int64_t, Req*> finished;
  std::deque<int64_t> done_q;
  int active_atoms = 0;
  int undelivered = 0;  // admitted, result not yet handed to the host
  RetireSlot slots[kRetireSlots];
  std::deque<int> inflight;  // retire slots in flight, oldest first
  // statistics (nnp_server_stats)
  int64_t rounds = 0, mixed_rounds = 0, max_phases = 0, peak_atoms = 0, retire_waits = 0;
  ~nnp_server() {
    // a request whose last step has run is owned by its retire slot until its
    // results arrive, then by the finished map
    for (Req* r : pending) delete r;
    for (Req* r : active)
      if (r->k <= r->n_steps) delete r;
    for (int q : inflight)
      for (auto& f : slots[q].reqs) delete f.first;
    for (auto& kv : finished) delete kv.second;
  }
};

namespace {

size_t server_state_bytes(int A, int M) {
  size_t b = 0;
  auto add = [&](size_t x) { b = align_up(b + x, 256); };
  add((size_t)A * 24); add((size_t)A * 24); add((size_t)A * 8); add((size_t)A * 4);
  add((size_t)A * 12); add((size_t)A * 12);
  add((size_t)(M + 1) * 4); add((size_t)M * 4); add((size_t)M * 4); add((size_t)M * 8);
  add((size_t)M * 8);
  add((size_t)A * 24); add((size_t)A * 24); add((size_t)A * 8); add((size_t)A * 4);
  add((size_t)A * 12); add((size_t)A * 4);
  add((size_t)A * 24); add((size_t)A * 24); add((size_t)A * 8); add((size_t)A * 4);
  add((size_t)M * 8);
  return b;
}

nnp_status status_from_bits(uint32_t word) {
  if (word & kStOffsets) return NNP_E_INVALID;
  if (word & kStSpecies) return NNP_E_SPECIES;
  if (word & kStNonFinite) return NNP_E_NONFINITE;
  if (word & kStCapacity) return NNP_E_CAPACITY;
  return NNP_OK;
}

// Hands the results of retire slot q (whose copies have completed) to the
// host side: status bits to the requests that were exposed to them, states
// and energies to the finishing requests, which become pollable.
void retire_deliver(nnp_server* s, int q) {
  RetireSlot& sl = s->slots[q];
  uint32_t word = 0;
  std::memcpy(&word, sl.h + sl.eo + 2 * (size_t)sl.nact, 4);
  if (word)
    for (Req* r : sl.exposed) r->status |= word;
  const double now = now_s();
  for (size_t k = 0; k < sl.reqs.size(); ++k) {
    Req* r = sl.reqs[k].first;
    const double* hx = sl.h + sl.reqs[k].second;
    r->x.assign(hx, hx + 3 * (size_t)r->n);
    r->v.assign(hx + 3 * r->n, hx + 6 * (size_t)r->n);
    r->e_pot = sl.h[sl.eo + sl.mol[k]];
    r->e_kin = sl.h[sl.eo + sl.nact + sl.mol[k]];
    r->t_done = now;
    s->finished[r->id] = r;
    s->done_q.push_back(r->id);
    --s->undelivered;
  }
  sl.reqs.clear();
  sl.mol.clear();
  sl.exposed.clear();
}

// Delivers the in-flight retire slots in order: those whose copies have
// completed, or (wait) all of them.
nnp_status retire_drain(nnp_server* s, bool wait) {
  while (!s->inflight.empty()) {
    const int q = s->inflight.front();
    if (wait) {
      if (hipEventSynchronize(s->slots[q].ev) != hipSuccess) return NNP_E_HIP;
    } else {
      const hipError_t e = hipEventQuery(s->slots[q].ev);
      if (e == hipErrorNotReady) {
        (void)hipGetLastError();  // the runtime records it as the last error
        break;
      }
      if (e != hipSuccess) return NNP_E_HIP;
    }
    retire_deliver(s, q);
    s->inflight.pop_front();
  }
  return NNP_OK;
}

// One MD step of the packed batch: forces at x, integration by per-molecule
// phase, kinetic energies, counters.  Every kernel reads the live atom and
// molecule counts from the workspace, so the same launches (or their graph)
// serve any batch up to the capacity.
nnp_status server_enqueue_step(nnp_server* s) {
  nnp_handle* h = s->h;
  const Plan& P = s->P;
  int* dims = at<int>(s->ws, P.dims);
  EvalIO io{-1, -1, nullptr, s->x, s->sp, s->off, s->epot, s->F, 1.f, nullptr, nullptr};
  io.keep_status = true;  // cleared when the retire copies read it
  nnp_status r = run(h, P, s->ws, io, s->st);
  if (r != NNP_OK) return r;
  if (s->lfm)
    launch_serve_lfm(dims, s->max_atoms, at<int>(s->ws, P.mol), s->off, s->kdone, s->nsteps,
                     s->seed, s->x, s->v, s->F, s->m, s->dt, s->lfm_c, s->lfm_kT, s->st);
  else
    launch_serve_integrate(dims, s->max_atoms, at<int>(s->ws, P.mol), s->kdone, s->nsteps, s->x,
                           s->v, s->F, s->m, s->dt, s->st);
  launch_kinetic(dims, s->max_mols, s->off, s->v, s->m, s->ekin, s->kdone, s->st);
  return launches_ok() ? NNP_OK : NNP_E_HIP;
}

}  // namespace

extern "C" {

nnp_status nnp_server_create(nnp_handle* h, size_t budget, int32_t max_atoms, int32_t max_mols,
                             double dt_fs, const double* mass_amu, void* stream,
                             nnp_server** out) {
  (void)stream;
  if (!h || !out || !mass_amu || max_atoms < 1 || max_mols < 1 || !(dt_fs > 0.0))
    return NNP_E_INVALID;
  *out = nullptr;
  if (hipSetDevice(h->device) != hipSuccess) return NNP_E_HIP;
  // fit the capacity to the HBM budget: state + workspace at capacity
  BoxConst B;
  make_box(h, nullptr, B);
  int A = max_atoms;
  for (;;) {
    const size_t need = server_state_bytes(A, max_mols) + make_plan(h, A, max_mols, B).total;
    if (need <= budget) break;
    const int A2 = (int)((double)A * (double)budget / (double)need * 0.98);
    if (A2 < 1 || A2 >= A) return NNP_E_OOM;
    A = A2;
  }
  nnp_server* s = new (std::nothrow) nnp_server();
  if (!s) return NNP_E_OOM;
  s->h = h;
  s->device = h->device;
  s->dt = dt_fs;
  for (int q = 0; q < h->S; ++q) s->mass_tab[q] = mass_amu[q];
  s->max_atoms = A;
  s->max_mols = max_mols;
  s->P = make_plan(h, A, max_mols, B);
  const size_t sb = server_state_bytes(A, max_mols);
  s->bytes = sb + s->P.total;
  if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&s->dmem, s->bytes) != hipSuccess) {
    if (s->st) (void)hipStreamDestroy(s->st);
    delete s;
    return NNP_E_OOM;
  }
  size_t o = 0;
  auto take = [&](size_t x) {
    char* p = s->dmem + o;
    o = align_up(o + x, 256);
    return p;
  };
  s->x = (double*)take((size_t)A * 24);
  s->v = (double*)take((size_t)A * 24);
  s->m = (double*)take((size_t)A * 8);
  s->sp = (int*)take((size_t)A * 4);
  s->F = (float*)take((size_t)A * 12);
  s->pos32 = (float*)take((size_t)A * 12);
  s->off = (int*)take((size_t)(max_mols + 1) * 4);
  s->kdone = (int*)take((size_t)max_mols * 4);
  s->nsteps = (int*)take((size_t)max_mols * 4);
  s->epot = (double*)take((size_t)max_mols * 8);
  s->ekin = (double*)take((size_t)max_mols * 8);
  s->x2 = (double*)take((size_t)A * 24);
  s->v2 = (double*)take((size_t)A * 24);
  s->m2 = (double*)take((size_t)A * 8);
  s->sp2 = (int*)take((size_t)A * 4);
  s->F2 = (float*)take((size_t)A * 12);
  s->src = (int*)take((size_t)A * 4);
  s->in_x = (double*)take((size_t)A * 24);
  s->in_v = (double*)take((size_t)A * 24);
  s->in_m = (double*)take((size_t)A * 8);
  s->in_sp = (int*)take((size_t)A * 4);
  s->seed = (uint64_t*)take((size_t)max_mols * 8);
  s->ws = s->dmem + align_up(sb, 256);
  // pinned host mirrors
  // src, in_sp | off, kdone, nsteps | dims | in_x, in_v, in_m | out (x, v, energies)
  const size_t slot_bytes = align_up((size_t)A * 48 + (size_t)max_mols * 16 + 16, 64);
  const size_t hb = (size_t)A * 8 + (size_t)(max_mols + 1) * 12 + 64 + (size_t)A * 56 +
                    (size_t)A * 48 + (size_t)max_mols * 24 + 4096 + kRetireSlots * slot_bytes;
  if (hipHostMalloc((void**)&s->hmem, hb) != hipSuccess) {
    (void)hipFree(s->dmem);
    (void)hipStreamDestroy(s->st);
    delete s;
    return NNP_E_OOM;
  }
  size_t ho = 0;
  auto htake = [&](size_t x) {
    char* p = s->hmem + ho;
    ho = align_up(ho + x, 64);
    return p;
  };
  s->h_src = (int*)htake((size_t)A * 4);
  s->h_in_sp = (int*)htake((size_t)A * 4);
  s->h_off = (int*)htake((size_t)(max_mols + 1) * 4);
  s->h_kdone = (int*)htake((size_t)max_mols * 4);
  s->h_nsteps = (int*)htake((size_t)max_mols * 4);
  s->h_dims = (int*)htake(16);
  s->h_in_x = (double*)htake((size_t)A * 24);
  s->h_in_v = (double*)htake((size_t)A * 24);
  s->h_in_m = (double*)htake((size_t)A * 8);
  s->h_out = (double*)htake((size_t)A * 48 + (size_t)max_mols * 16);
  s->h_seed = (uint64_t*)htake((size_t)max_mols * 8);
  bool evs = hip_ok(hipEventCreateWithFlags(&s->ev_upload, hipEventDisableTiming));
  for (int q = 0; q < kRetireSlots; ++q) {
    s->slots[q].h = (double*)htake(slot_bytes);
    evs &= hip_ok(hipEventCreateWithFlags(&s->slots[q].ev, hipEventDisableTiming));
  }
  if (!evs) {
    nnp_server_destroy(s);
    return NNP_E_HIP;
  }
  // empty batch: counts 0, offsets {0}
  s->h_dims[0] = 0;
  s->h_dims[1] = 0;
  s->h_off[0] = 0;
  launch_fill_i32(reinterpret_cast<int*>(at<uint32_t>(s->ws, s->P.status)), 0, 1, s->st);
  bool ok = hip_ok(hipMemcpyAsync(at<int>(s->ws, s->P.dims), s->h_dims, 8, hipMemcpyHostToDevice,
                                  s->st)) &&
            hip_ok(hipMemcpyAsync(s->off, s->h_off, 4, hipMemcpyHostToDevice, s->st)) &&
            hip_ok(hipStreamSynchronize(s->st));
  if (!ok) {
    nnp_server_destroy(s);
    return NNP_E_HIP;
  }
  *out = s;
  return NNP_OK;
}

void nnp_server_destroy(nnp_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  if (s->ev_upload) (void)hipEventDestroy(s->ev_upload);
  for (int q = 0; q < kRetireSlots; ++q)
    if (s->slots[q].ev) (void)hipEventDestroy(s->slots[q].ev);
  if (s->hmem) (void)hipHostFree(s->hmem);
  if (s->dmem) (void)hipFree(s->dmem);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

nnp_status nnp_server_submit(nnp_server* s, int64_t id, int32_t n, const double* x,
                             const double* v, const int32_t* species, int32_t n_steps) {
  if (!s || n < 1 || !x || !v || !species || n_steps < 1) return NNP_E_INVALID;
  if (n > s->max_atoms) return NNP_E_BUSY;
  for (int i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= s->h->S) return NNP_E_SPECIES;
  Req* r = new (std::nothrow) Req();
  if (!r) return NNP_E_OOM;
  r->id = id;
  r->n = n;
  r->n_steps = n_steps;
  r->x.assign(x, x + 3 * (size_t)n);
  r->v.assign(v, v + 3 * (size_t)n);
  r->sp.assign(species, species + n);
  r->t_submit = now_s();
  s->pending.push_back(r);
  return NNP_OK;
}

nnp_status nnp_server_set_langevin(nnp_server* s, double temperature, double friction) {
  if (!s || !(temperature >= 0.0) || !(friction >= 0.0)) return NNP_E_INVALID;
  // the integrator is part of the captured step: fixed before the first step
  if (s->warmed || !s->active.empty()) return NNP_E_INVALID;
  s->lfm = true;
  s->lfm_c = std::exp(-friction * 1e-3 * s->dt);
  s->lfm_kT = 8.617333262e-5 * temperature * 9.648533e-3;
  return NNP_OK;
}

int32_t nnp_server_active(const nnp_server* s) { return s ? (int32_t)s->undelivered : 0; }
int32_t nnp_server_pending(const nnp_server* s) { return s ? (int32_t)s->pending.size() : 0; }

nnp_status nnp_server_step(nnp_server* s) {
  if (!s) return NNP_E_INVALID;
  if (hipSetDevice(s->h->device) != hipSuccess) return NNP_E_HIP;
  // 0. results whose copies have arrived
  nnp_status rs = retire_drain(s, false);
  if (rs != NNP_OK) return rs;
  // 1. drop requests whose final step ran in the previous round
  std::vector<Req*> keep;
  bool changed = false;
  for (Req* r : s->active) {
    if (r->k > r->n_steps) {
      changed = true;
      s->active_atoms -= r->n;
    } else {
      keep.push_back(r);
    }
  }
  // 2. admit in arrival order while atoms and molecule slots allow
  std::vector<Req*> admit;
  int atoms = s->active_atoms;
  int mols = (int)keep.size();
  while (!s->pending.empty()) {
    Req* r = s->pending.front();
    if (atoms + r->n > s->max_atoms || mols + 1 > s->max_mols) break;
    s->pending.pop_front();
    admit.push_back(r);
    atoms += r->n;
    ++mols;
  }
  if (!admit.empty()) changed = true;
  if (!admit.empty() && !keep.empty()) ++s->mixed_rounds;
  s->undelivered += (int)admit.size();
  // 3. repack on the device: survivors keep their state, admitted atoms come
  //    from staging
  if (changed) {
    if (hipEventSynchronize(s->ev_upload) != hipSuccess) return NNP_E_HIP;
    std::vector<int> old_start(s->active.size());
    {
      int o = 0;
      for (size_t q = 0; q < s->active.size(); ++q) {
        old_start[q] = o;
        o += s->active[q]->n;
      }
    }
    int t = 0, mcount = 0, staged = 0;
    s->h_off[0] = 0;
    size_t aq = 0;
    for (size_t q = 0; q < s->active.size(); ++q) {
      Req* r = s->active[q];
      if (r->k > r->n_steps) continue;
      for (int i = 0; i < r->n; ++i) s->h_src[t++] = old_start[q] + i;
      s->h_kdone[mcount] = r->k;
      s->h_nsteps[mcount] = r->n_steps;
      s->h_seed[mcount] = (uint64_t)r->id;
      s->h_off[++mcount] = t;
      ++aq;
    }
    const double now = now_s();
    for (Req* r : admit) {
      for (int i = 0; i < r->n; ++i) {
        s->h_src[t++] = -(staged + i) - 1;
        for (int c = 0; c < 3; ++c) {
          s->h_in_x[3 * (staged + i) + c] = r->x[3 * i + c];
          s->h_in_v[3 * (staged + i) + c] = r->v[3 * i + c];
        }
        s->h_in_sp[staged + i] = r->sp[i];
        s->h_in_m[staged + i] = s->mass_tab[r->sp[i]];
      }
      staged += r->n;
      r->k = 0;
      r->t_admit = now;
      s->h_kdone[mcount] = 0;
      s->h_nsteps[mcount] = r->n_steps;
      s->h_seed[mcount] = (uint64_t)r->id;
      s->h_off[++mcount] = t;
    }
    s->h_dims[0] = t;
    s->h_dims[1] = mcount;
    hipStream_t st = s->st;
    bool ok = true;
    if (staged) {
      ok &= hip_ok(hipMemcpyAsync(s->in_x, s->h_in_x, (size_t)staged * 24, hipMemcpyHostToDevice, st));
      ok &= hip_ok(hipMemcpyAsync(s->in_v, s->h_in_v, (size_t)staged * 24, hipMemcpyHostToDevice, st));
      ok &= hip_ok(hipMemcpyAsync(s->in_m, s->h_in_m, (size_t)staged * 8, hipMemcpyHostToDevice, st));
      ok &= hip_ok(hipMemcpyAsync(s->in_sp, s->h_in_sp, (size_t)staged * 4, hipMemcpyHostToDevice, st));
    }
    if (t) ok &= hip_ok(hipMemcpyAsync(s->src, s->h_src, (size_t)t * 4, hipMemcpyHostToDevice, st));
    ok &= hip_ok(hipMemcpyAsync(s->off, s->h_off, (size_t)(mcount + 1) * 4, hipMemcpyHostToDevice, st));
    if (mcount) {
      ok &= hip_ok(hipMemcpyAsync(s->kdone, s->h_kdone, (size_t)mcount * 4, hipMemcpyHostToDevice, st));
      ok &= hip_ok(hipMemcpyAsync(s->nsteps, s->h_nsteps, (size_t)mcount * 4, hipMemcpyHostToDevice, st));
      ok &= hip_ok(hipMemcpyAsync(s->seed, s->h_seed, (size_t)mcount * 8, hipMemcpyHostToDevice, st));
    }
    ok &= hip_ok(hipMemcpyAsync(at<int>(s->ws, s->P.dims), s->h_dims, 8, hipMemcpyHostToDevice, st));
    ok &= hip_ok(hipEventRecord(s->ev_upload, st));
    if (!ok) return NNP_E_HIP;
    launch_gather_rows(s->src, t, s->x, s->v, s->sp, s->m, s->F, s->in_x, s->in_v, s->in_sp,
                       s->in_m, s->x2, s->v2, s->sp2, s->m2, s->F2, st);
    ok &= hip_ok(hipMemcpyAsync(s->x, s->x2, (size_t)t * 24, hipMemcpyDeviceToDevice, st));
    ok &= hip_ok(hipMemcpyAsync(s->v, s->v2, (size_t)t * 24, hipMemcpyDeviceToDevice, st));
    ok &= hip_ok(hipMemcpyAsync(s->m, s->m2, (size_t)t * 8, hipMemcpyDeviceToDevice, st));
    ok &= hip_ok(hipMemcpyAsync(s->sp, s->sp2, (size_t)t * 4, hipMemcpyDeviceToDevice, st));
    if (!ok) return NNP_E_HIP;
    std::vector<Req*> next;
    for (Req* r : keep) next.push_back(r);
    for (Req* r : admit) next.push_back(r);
    s->active.swap(next);
    s->active_atoms = atoms;
  }
  if (s->active.empty()) return retire_drain(s, true);  // nothing to run: wait for results
  {
    // statistics: atoms on the device, distinct step counters in one launch
    std::vector<int> ks;
    for (Req* q : s->active) ks.push_back(q->k);
    std::sort(ks.begin(), ks.end());
    const int64_t phases = std::unique(ks.begin(), ks.end()) - ks.begin();
    s->max_phases = std::max(s->max_phases, phases);
    s->peak_atoms = std::max<int64_t>(s->peak_atoms, s->active_atoms);
    ++s->rounds;
  }
  // 4. one step over the whole batch (graph replay after a first eager step)
  nnp_status r;
  if (!s->warmed) {
    r = server_enqueue_step(s);
    if (r != NNP_OK) return r;
    s->warmed = true;
  } else {
    if (!s->exec) {
      if (hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return NNP_E_HIP;
      r = server_enqueue_step(s);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(s->st, &g);
      if (r != NNP_OK || ec != hipSuccess) return r != NNP_OK ? r : NNP_E_HIP;
      s->graph = g;
      if (hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0) != hipSuccess) return NNP_E_HIP;
    }
    if (hipGraphLaunch(s->exec, s->st) != hipSuccess) return NNP_E_HIP;
  }
  for (Req* q : s->active) q->k += 1;
  // 5. requests whose closing half kick ran: copy their results, the batch's
  //    energies and the status word to a pinned retire slot behind an event;
  //    a later round hands them over
  std::vector<std::pair<Req*, int>> fin;  // request, first atom in the batch
  std::vector<int> fin_mol;
  {
    int o = 0, mi = 0;
    for (Req* q : s->active) {
      if (q->k > q->n_steps) {
        fin.push_back({q, o});
        fin_mol.push_back(mi);
      }
      o += q->n;
      ++mi;
    }
  }
  if (!fin.empty()) {
    if ((int)s->inflight.size() == kRetireSlots) {  // every slot busy: wait for the oldest
      const int q = s->inflight.front();
      if (hipEventSynchronize(s->slots[q].ev) != hipSuccess) return NNP_E_HIP;
      retire_deliver(s, q);
      s->inflight.pop_front();
      ++s->retire_waits;
    }
    int q = 0;
    while (std::find(s->inflight.begin(), s->inflight.end(), q) != s->inflight.end()) ++q;
    RetireSlot& sl = s->slots[q];
    size_t ho = 0;
    bool ok = true;
    for (size_t k = 0; k < fin.size(); ++k) {
      Req* r = fin[k].first;
      const size_t nb = (size_t)r->n * 24;
      ok &= hip_ok(hipMemcpyAsync(sl.h + ho, s->x + 3 * (size_t)fin[k].second, nb,
                                  hipMemcpyDeviceToHost, s->st));
      ok &= hip_ok(hipMemcpyAsync(sl.h + ho + 3 * r->n, s->v + 3 * (size_t)fin[k].second, nb,
                                  hipMemcpyDeviceToHost, s->st));
      sl.reqs.push_back({r, ho});
      sl.mol.push_back(fin_mol[k]);
      ho += 6 * (size_t)r->n;
    }
    sl.nact = (int)s->active.size();
    sl.eo = ho;
    ok &= hip_ok(hipMemcpyAsync(sl.h + ho, s->epot, (size_t)sl.nact * 8, hipMemcpyDeviceToHost,
                                s->st));
    ok &= hip_ok(hipMemcpyAsync(sl.h + ho + sl.nact, s->ekin, (size_t)sl.nact * 8,
                                hipMemcpyDeviceToHost, s->st));
    uint32_t* status = at<uint32_t>(s->ws, s->P.status);
    ok &= hip_ok(hipMemcpyAsync(sl.h + ho + 2 * (size_t)sl.nact, status, 4,
                                hipMemcpyDeviceToHost, s->st));
    launch_fill_i32(reinterpret_cast<int*>(status), 0, 1, s->st);  // the next rounds' bits
    sl.exposed = s->active;
    ok &= hip_ok(hipEventRecord(sl.ev, s->st));
    if (!ok) return NNP_E_HIP;
    s->inflight.push_back(q);
  }
  return NNP_OK;
}

int32_t nnp_server_poll(nnp_server* s, int64_t* ids, int32_t max) {
  if (!s || !ids || max < 1) return 0;
  (void)retire_drain(s, false);
  int32_t k = 0;
  while (k < max && !s->done_q.empty()) {
    ids[k++] = s->done_q.front();
    s->done_q.pop_front();
  }
  return k;
}

nnp_status nnp_server_result(nnp_server* s, int64_t id, double* x, double* v, double* e_pot,
                             double* e_kin, double* t_submit, double* t_admit, double* t_done) {
  if (!s) return NNP_E_INVALID;
  auto it = s->finished.find(id);
  if (it == s->finished.end()) return NNP_E_INVALID;
  Req* r = it->second;
  if (x) std::memcpy(x, r->x.data(), r->x.size() * 8);
  if (v) std::memcpy(v, r->v.data(), r->v.size() * 8);
  if (e_pot) *e_pot = r->e_pot;
  if (e_kin) *e_kin = r->e_kin;
  if (t_submit) *t_submit = r->t_submit;
  if (t_admit) *t_admit = r->t_admit;
  if (t_done) *t_done = r->t_done;
  return status_from_bits(r->status);
}

nnp_status nnp_server_stats(const nnp_server* s, int64_t* out, int32_t n) {
  if (!s || !out || n < 1) return NNP_E_INVALID;
  const int64_t v[8] = {s->max_atoms, s->max_mols, s->active_atoms, s->peak_atoms,
                        s->rounds,    s->mixed_rounds, s->max_phases, s->retire_waits};
  for (int32_t k = 0; k < n && k < 8; ++k) out[k] = v[k];
  return NNP_OK;
}

}  // extern "C"

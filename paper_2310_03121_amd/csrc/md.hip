// Velocity-Verlet and LF-Middle Langevin integration (FP64 state, FP32
// forces) and the device-side repacking used by the continuous-batching
// server.
//
// Units: A, fs, amu, eV; a = 9.648533e-3 * F / m in A/fs^2.  The positions fed
// to the potential are the FP32 rounding of the FP64 positions.
//
// The server advances every active molecule with one force evaluation per
// step.  A molecule's step is driven by its per-molecule counter k (steps
// done) and its step count n:
//   k == 0      : v += dt/2 a(x);            x += dt v       (first half kick)
//   0 < k < n   : v += dt   a(x);            x += dt v       (closing half kick
//                                                             of the previous
//                                                             step + opening
//                                                             half kick)
//   k == n      : v += dt/2 a(x)                             (closing half kick)
// which is velocity Verlet with the force at each x evaluated once.
#include "kernels.h"

namespace nnp {

constexpr double kAccUnit = 9.648533e-3;

__global__ __launch_bounds__(256) void k_vv_kick_drift(const int* __restrict__ dims, double* __restrict__ x,
                                                       double* __restrict__ v, const float* __restrict__ F,
                                                       const double* __restrict__ mass, double dt,
                                                       float* __restrict__ pos32) {
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 0.5 * dt * kAccUnit / mass[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double vv = v[3 * i + c] + s * (double)F[3 * i + c];
    const double xx = x[3 * i + c] + dt * vv;
    v[3 * i + c] = vv;
    x[3 * i + c] = xx;
    pos32[3 * i + c] = (float)xx;
  }
}

__global__ __launch_bounds__(256) void k_vv_kick(const int* __restrict__ dims, double* __restrict__ v,
                                                 const float* __restrict__ F,
                                                 const double* __restrict__ mass, double dt) {
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 0.5 * dt * kAccUnit / mass[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) v[3 * i + c] += s * (double)F[3 * i + c];
}

// ---------------------------------------------------------- LF-Middle Langevin
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC '11): 128-bit counter, 64-bit
// key, ten rounds of two 32x32->64 multiplies by fixed odd constants with
// the high halves folded into the other words and the key; Weyl increments
// bump the key between rounds.  Written from the published definition.
struct Philox4 {
  uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kM0, c0), lo0 = kM0 * c0;
    const uint32_t hi1 = __umulhi(kM1, c2), lo1 = kM1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kW0;
    k1 += kW1;
  }
  return Philox4{{c0, c1, c2, c3}};
}

// Box-Muller in FP64 over two 32-bit words: u = (wa + 1) 2^-32 in (0, 1],
// theta = 2 pi wb 2^-32.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& n0, double& n1) {
  const double u = ((double)wa + 1.0) * 0x1p-32;
  const double th = 6.283185307179586477 * (double)wb * 0x1p-32;
  const double r = sqrt(-2.0 * log(u));
  double s, c;
  sincos(th, &s, &c);
  n0 = r * c;
  n1 = r * s;
}

// One LF-Middle step for every atom (x_n, v_{n-1/2}, F(x_n) -> x_{n+1},
// v_{n+1/2}):  v += dt a;  x += dt/2 v;  v = c v + sqrt((1 - c^2) kB T / m) R;
// x += dt/2 v.  R: the first three normals of Philox block (atom, step lo,
// step hi, 0) under key (seed lo, seed hi).  kT_acc = kB T * (A/fs^2 per
// eV/A/amu), so kT_acc / m is the velocity variance in A^2/fs^2.
__device__ __forceinline__ void lfm_update(double* __restrict__ x, double* __restrict__ v,
                                           const float* __restrict__ F, double m, double dt,
                                           double c, double kT_acc, uint32_t ctr0, uint64_t step,
                                           uint64_t seed, float* __restrict__ pos32) {
  const Philox4 w = philox4x32_10(ctr0, (uint32_t)step, (uint32_t)(step >> 32), 0u,
                                  (uint32_t)seed, (uint32_t)(seed >> 32));
  double R[4];
  box_muller(w.v[0], w.v[1], R[0], R[1]);
  box_muller(w.v[2], w.v[3], R[2], R[3]);
  const double s = dt * kAccUnit / m;
  const double sig = sqrt((1.0 - c * c) * kT_acc / m);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double vv = v[k] + s * (double)F[k];
    double xx = x[k] + 0.5 * dt * vv;
    vv = c * vv + sig * R[k];
    xx += 0.5 * dt * vv;
    v[k] = vv;
    x[k] = xx;
    if (pos32) pos32[k] = (float)xx;
  }
}

__global__ __launch_bounds__(256) void k_lfm_step(const int* __restrict__ dims,
                                                  double* __restrict__ x, double* __restrict__ v,
                                                  const float* __restrict__ F,
                                                  const double* __restrict__ mass, double dt,
                                                  double c, double kT_acc, uint64_t seed,
                                                  uint64_t step, float* __restrict__ pos32) {
  const int n = dims[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  lfm_update(x + 3 * i, v + 3 * i, F + 3 * i, mass[i], dt, c, kT_acc, (uint32_t)i, step, seed,
             pos32 + 3 * i);
}

// Server step, LF-Middle: a molecule with k < n steps done takes one step
// with its own noise stream (counter: the atom's index inside its molecule
// and the molecule's step k; key: the request's seed), so a request draws
// the same numbers alone and inside any batch; at k == n it waits to be
// retired with x_n and v_{n-1/2}.
__global__ __launch_bounds__(256) void k_serve_lfm(const int* __restrict__ dims,
                                                   const int* __restrict__ mol,
                                                   const int* __restrict__ off,
                                                   const int* __restrict__ kdone,
                                                   const int* __restrict__ nsteps,
                                                   const uint64_t* __restrict__ seed,
                                                   double* __restrict__ x, double* __restrict__ v,
                                                   const float* __restrict__ F,
                                                   const double* __restrict__ mass, double dt,
                                                   double c, double kT_acc) {
  const int n = dims[0], nmol = dims[1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = clampi(mol[i], nmol);
  const int k = kdone[m], ns = nsteps[m];
  if (k >= ns) return;
  lfm_update(x + 3 * i, v + 3 * i, F + 3 * i, mass[i], dt, c, kT_acc, (uint32_t)(i - off[m]),
             (uint64_t)k, seed[m], nullptr);
}

// Kinetic energy per molecule; with `kdone`, also advances the molecule's
// step counter (serving).
__global__ __launch_bounds__(256) void k_kinetic(const int* __restrict__ dims, const int* __restrict__ off,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ mass,
                                                 double* __restrict__ ke, int* __restrict__ kdone) {
  const int n = dims[0], nmol = dims[1];
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= nmol) return;
  int a = off[m], b = off[m + 1];
  a = a < 0 ? 0 : (a > n ? n : a);
  b = b < a ? a : (b > n ? n : b);
  double acc = 0.0;
  for (int i = a + lane_id(); i < b; i += kWave)
    acc += mass[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
  acc = wave_sum_d(acc);
  if (lane_id() == 0) {
    ke[m] = 0.5 * acc / kAccUnit;
    if (kdone) kdone[m] += 1;
  }
}

// Server step integration, driven by per-molecule counters (see above).
__global__ __launch_bounds__(256) void k_serve_integrate(const int* __restrict__ dims,
                                                         const int* __restrict__ mol,
                                                         const int* __restrict__ kdone,
                                                         const int* __restrict__ nsteps,
                                                         double* __restrict__ x, double* __restrict__ v,
                                                         const float* __restrict__ F,
                                                         const double* __restrict__ mass, double dt) {
  const int n = dims[0], nmol = dims[1];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = clampi(mol[i], nmol);
  const int k = kdone[m], ns = nsteps[m];
  if (k > ns) return;  // finished, waiting to be retired
  const double kick = (k == 0 || k == ns) ? 0.5 * dt : dt;
  const bool drift = k < ns;
  const double s = kick * kAccUnit / mass[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double vv = v[3 * i + c] + s * (double)F[3 * i + c];
    v[3 * i + c] = vv;
    if (drift) x[3 * i + c] += dt * vv;
  }
}

// New packed atom t takes its state from old packed atom src[t] (>= 0) or from
// staging slot -src[t]-1 (newly admitted atoms).
__global__ __launch_bounds__(256) void k_gather_rows(const int* __restrict__ src, int n,
                                                     const double* __restrict__ x_old,
                                                     const double* __restrict__ v_old,
                                                     const int* __restrict__ sp_old,
                                                     const double* __restrict__ m_old,
                                                     const float* __restrict__ f_old,
                                                     const double* __restrict__ x_in,
                                                     const double* __restrict__ v_in,
                                                     const int* __restrict__ sp_in,
                                                     const double* __restrict__ m_in,
                                                     double* __restrict__ x, double* __restrict__ v,
                                                     int* __restrict__ sp, double* __restrict__ m,
                                                     float* __restrict__ f) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int s = src[t];
  if (s >= 0) {
    for (int c = 0; c < 3; ++c) {
      x[3 * t + c] = x_old[3 * s + c];
      v[3 * t + c] = v_old[3 * s + c];
      f[3 * t + c] = f_old[3 * s + c];
    }
    sp[t] = sp_old[s];
    m[t] = m_old[s];
  } else {
    const int q = -s - 1;
    for (int c = 0; c < 3; ++c) {
      x[3 * t + c] = x_in[3 * q + c];
      v[3 * t + c] = v_in[3 * q + c];
      f[3 * t + c] = 0.f;
    }
    sp[t] = sp_in[q];
    m[t] = m_in[q];
  }
}

// ----------------------------------------------------------------- launchers

void launch_vv_kick_drift(const int* dims, int n_cap, double* x, double* v, const float* F,
                          const double* mass, double dt, float* pos32, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_vv_kick_drift, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, x, v, F,
                     mass, dt, pos32);
}

void launch_vv_kick(const int* dims, int n_cap, double* v, const float* F, const double* mass,
                    double dt, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_vv_kick, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, v, F, mass, dt);
}

void launch_lfm_step(const int* dims, int n_cap, double* x, double* v, const float* F,
                     const double* mass, double dt, double c, double kT_acc, uint64_t seed,
                     uint64_t step, float* pos32, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_lfm_step, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, x, v, F, mass,
                     dt, c, kT_acc, seed, step, pos32);
}

void launch_serve_lfm(const int* dims, int n_cap, const int* mol, const int* off,
                      const int* kdone, const int* nsteps, const uint64_t* seed, double* x,
                      double* v, const float* F, const double* mass, double dt, double c,
                      double kT_acc, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_serve_lfm, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, mol, off,
                     kdone, nsteps, seed, x, v, F, mass, dt, c, kT_acc);
}

void launch_kinetic(const int* dims, int nmol_cap, const int* off, const double* v,
                    const double* mass, double* ke, int* kdone, hipStream_t st) {
  if (nmol_cap <= 0) return;
  hipLaunchKernelGGL(k_kinetic, dim3((nmol_cap + 3) / 4), dim3(256), 0, st, dims, off, v, mass, ke,
                     kdone);
}

void launch_serve_integrate(const int* dims, int n_cap, const int* mol, const int* kdone,
                            const int* nsteps, double* x, double* v, const float* F,
                            const double* mass, double dt, hipStream_t st) {
  if (n_cap <= 0) return;
  hipLaunchKernelGGL(k_serve_integrate, dim3((n_cap + 255) / 256), dim3(256), 0, st, dims, mol,
                     kdone, nsteps, x, v, F, mass, dt);
}

void launch_gather_rows(const int* src, int n, const double* x_old, const double* v_old,
                        const int* sp_old, const double* m_old, const float* f_old,
                        const double* x_in, const double* v_in, const int* sp_in,
                        const double* m_in, double* x, double* v, int* sp, double* m, float* f,
                        hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((n + 255) / 256), dim3(256), 0, st, src, n, x_old, v_old,
                     sp_old, m_old, f_old, x_in, v_in, sp_in, m_in, x, v, sp, m, f);
}

}  // namespace nnp

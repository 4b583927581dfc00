// Velocity-Verlet integration (FP64 state, FP32 forces) and the device-side
// repacking used by the continuous-batching server.
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

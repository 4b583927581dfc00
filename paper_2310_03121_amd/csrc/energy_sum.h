// The molecular energy sum as one workgroup's work, shared by the energy
// kernel and the adjoint launch that runs it beside the force scatter.
#pragma once
#include "kernels.h"

namespace nnp {

struct EnergyArgs {
  const int* off;          // molecule offsets [nmol + 1]
  const float4* xyzs;      // staged records (species in .w)
  const float* eatom;      // atomic energies, input atom order; member k at + k * mstride
  int n_models;
  long mstride;
  const double* eself;     // [kMaxS]
  double* E;               // [nmol]; null: no energy sum
  uint32_t* status;
};

// One workgroup (256 threads or more; the first 256 do the sums) per molecule m: E_m = sum_i (e_i + e_self[s_i])
// with the atomic energies in input atom order; for an ensemble of M members
// e_i is the mean of the members' atomic energies.  Thread t sums the atoms
// t, t + 256, ... of the molecule (counted from its first atom), then the
// waves and the four wave sums combine in a fixed order: the result depends
// only on the molecule's own atoms, not on where it sits in a batch.
__device__ __forceinline__ void energy_block(int m, const int* __restrict__ dims,
                                             const EnergyArgs& A) {
  const int* __restrict__ off = A.off;
  const float4* __restrict__ xyzs = A.xyzs;
  const float* __restrict__ eatom = A.eatom;
  const int n_models = A.n_models;
  const long mstride = A.mstride;
  const double* __restrict__ eself = A.eself;
  double* __restrict__ E = A.E;
  uint32_t* __restrict__ status = A.status;
  __shared__ double part[4];
  __shared__ double es[kMaxS];  // self energies: no dependent global gather per atom
  const int n = dims[0], nmol = dims[1];
  if (m >= nmol) return;
  if (threadIdx.x < kMaxS) es[threadIdx.x] = eself[threadIdx.x];
  __syncthreads();
  int a = off[m], b = off[m + 1];
  a = a < 0 ? 0 : (a > n ? n : a);
  b = b < a ? a : (b > n ? n : b);
  double acc = 0.0;
  // the first 256 threads sum, whatever the workgroup size, so that the
  // order of the additions (and so the result) is the same in every launch
  const int nt = threadIdx.x < 256 ? 256 : 0;
  if (n_models == 1) {  // straight-line loop body: loads of several atoms in flight
#pragma unroll 4
    for (int i = a + (int)threadIdx.x; i < b && nt; i += 256)
      acc += (double)eatom[i] + es[__float_as_int(xyzs[i].w) & (kMaxS - 1)];
  } else {
    const double inv_m = 1.0 / n_models;
    for (int i = a + (int)threadIdx.x; i < b && nt; i += 256) {
      double e = (double)eatom[i];
      for (int k = 1; k < n_models; ++k) e += (double)eatom[k * mstride + i];
      acc += e * inv_m + es[__float_as_int(xyzs[i].w) & (kMaxS - 1)];
    }
  }
  acc = wave_sum_d(acc);
  if (lane_id() == 0 && threadIdx.x < 256) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double e = ((part[0] + part[1]) + part[2]) + part[3];
    E[m] = e;
    if (!isfinite(e)) atomicOr(status, kStNonFinite);
  }
}

}  // namespace nnp

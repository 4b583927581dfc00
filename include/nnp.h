/*
 * nnp.h -- C ABI of the MI355X (gfx950) engine for ANI-style symmetry-function
 * neural network potentials: energies, forces, parameter gradients and
 * velocity-Verlet MD serving.
 *
 * The operations are those the OpenMM 8 paper names for machine-learning
 * potentials: a model maps atomic positions to a potential energy and forces
 * follow by backpropagation (Methods, "PyTorch Model Support"); the ANI
 * potentials use one network per element (Methods, "OpenMM-ML": seven elements
 * for ANI-2x, four for ANI-1ccx); the expensive steps are building neighbor
 * lists and computing the ANI atom-centered symmetry functions (Methods,
 * "Optimization Through NNPOps").  The symmetry functions are the published
 * ANI definition (radial and angular terms with a cosine cutoff); the paper
 * benchmarks the ANI-2x model inside MD (Results, Table 3).
 *
 * Conventions shared by every entry point:
 *   - Units: A (positions), eV (energies), eV/A (forces), amu, fs.
 *   - Pointers documented "device" must point to device memory on the current
 *     HIP device; "host" pointers to ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Entry points that take a stream only enqueue work; they never
 *     synchronise unless stated.
 *   - Host-checkable errors return synchronously and enqueue nothing.
 *     Errors that only the device can see (species out of range, non-finite
 *     positions or energies, neighbor-list overflow, malformed molecule
 *     offsets) set bits of a status word in the workspace; read it with
 *     nnp_check() after the stream has run.  Outputs are undefined while such
 *     a bit is set.  Kernels clamp every data-derived index, so a bad input
 *     never makes them access memory out of bounds.
 *   - No entry point throws; none aborts.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnp_handle nnp_handle;
typedef struct nnp_server nnp_server;

typedef enum {
  NNP_OK = 0,
  NNP_E_INVALID = 1,   /* bad argument (null pointer, count, layout, offsets) */
  NNP_E_SPECIES = 2,   /* species index outside [0, n_species)               */
  NNP_E_BOX = 3,       /* a box edge is shorter than twice the radial cutoff  */
  NNP_E_CAPACITY = 4,  /* an atom has more neighbors than the list holds     */
  NNP_E_OOM = 5,       /* device allocation failed (nnp_create, servers)     */
  NNP_E_HIP = 6,       /* a HIP runtime call failed                          */
  NNP_E_NONFINITE = 7, /* non-finite position or energy                      */
  NNP_E_WORKSPACE = 8, /* workspace missing or smaller than required         */
  NNP_E_BUSY = 9       /* server: no capacity for the request right now      */
} nnp_status;

typedef enum {
  NNP_MLP_FP32 = 0, /* networks in FP32 on MFMA, FP32 accumulation           */
  NNP_MLP_BF16 = 1  /* network operands BF16 on MFMA, FP32 accumulation      */
} nnp_precision;

/* Symmetry-function parameters (host memory; copied by nnp_create).
 * The engine supports the ANI layout: n_shf_r = 16, n_shf_a = 4, n_shf_z = 8,
 * 1 <= n_species <= 8.  One atom's feature vector G has
 * F = 16*S + 32*S*(S+1)/2 entries: radial block of neighbor species s at
 * 16*s + m; angular block of the unordered species pair (p <= q) at
 * 16*S + 32*P(p,q) + 8*a + z, P(p,q) = p*S - p*(p-1)/2 + (q - p).
 *   radial  : G[16*s_j + m] += c_R exp(-eta_r (d_ij - shf_r[m])^2) fc(d_ij; rc_rad)
 *   angular : over unordered neighbor pairs {j,k} within rc_ang,
 *             theta = acos(kappa cos(angle j-i-k)),
 *             G[...] += 2^(1-zeta) (1 + cos(theta - shf_z[z]))^zeta
 *                       exp(-eta_a ((d_ij + d_ik)/2 - shf_a[a])^2)
 *                       fc(d_ij; rc_ang) fc(d_ik; rc_ang)
 *   fc(d; R) = cos(pi d / R)/2 + 1/2 for d < R, 0 otherwise.
 * Neighbor sets use a float32 predicate evaluated without FMA contraction:
 * dx = fl(x_j - x_i) (minimum image with a box: dx -= L*rint(dx*fl(1/L))),
 * d2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)), neighbor iff same molecule,
 * j != i and d2 < fl(R*R). */
typedef struct {
  int32_t n_species;
  float rc_rad;
  float eta_r;
  int32_t n_shf_r;
  const float* shf_r;
  float rc_ang;
  float eta_a;
  float zeta;
  int32_t n_shf_a;
  const float* shf_a;
  int32_t n_shf_z;
  const float* shf_z;
  float radial_prefactor; /* c_R; the ANI-2x convention is 0.25 */
  float angle_cos_scale;  /* kappa in (0, 1); the ANI-2x convention is 0.95 */
} nnp_aev_params;

/* Per-element networks (host memory; copied and repacked by nnp_create).
 * Layer l maps width[l] -> width[l+1]; hidden layers apply
 * CELU_alpha(x) = max(0,x) + min(0, alpha (exp(x/alpha) - 1)); the last layer
 * is linear with width[n_layers] == 1.  The engine supports n_layers == 4 and
 * width[0] == F.  `params` is one float32 vector: for species s = 0..S-1, for
 * layer l = 0..n_layers-1: W_l (width[l+1] x width[l], row-major) then b_l.
 * The atomic energy is E_i = net_{s_i}(G_i) + self_energy[s_i]. */
typedef struct {
  int32_t n_layers;
  const int32_t* width;      /* n_layers + 1 entries */
  float celu_alpha;
  const float* params;       /* nnp_param_count() floats */
  const double* self_energy; /* n_species entries, or NULL for zeros */
} nnp_mlp_params;

/* Creates a potential on the current HIP device: validates the parameters,
 * uploads the symmetry-function constants and packs the weights (FP32 master
 * copy, BF16 copy and transposed copies for the adjoint).  This is the only
 * call that copies weights from the host.  Returns NNP_E_INVALID for an
 * unsupported layout, NNP_E_OOM / NNP_E_HIP on device failures. */
nnp_status nnp_create(const nnp_aev_params* aev, const nnp_mlp_params* mlp,
                      nnp_precision precision, nnp_handle** out);

/* An ensemble of n_models (1..8) independently trained networks over one set
 * of symmetry functions (Results, "Performance of MLPs": ANI-2x averages
 * eight models; Table 3 times the ensemble against a single member).
 * `mlps` is host memory, n_models entries with identical n_layers, widths
 * and celu_alpha (else NNP_E_INVALID); self energies are taken from mlps[0].
 * Every evaluation call then returns the ensemble mean: E_m is the mean of
 * the members' molecular energies and the forces are the mean of their
 * forces.  Neighbor lists and symmetry functions are computed once per
 * evaluation, the networks run member by member, and the members' dE/dG are
 * summed inside one product before the symmetry-function adjoint, which runs
 * once.  nnp_create(aev, mlp, p, out) is nnp_create_ensemble(aev, mlp, 1, p,
 * out).  Weight gradients (nnp_backward with dL_dparams) need n_models == 1. */
nnp_status nnp_create_ensemble(const nnp_aev_params* aev, const nnp_mlp_params* mlps,
                               int32_t n_models, nnp_precision precision, nnp_handle** out);
void nnp_destroy(nnp_handle* h);

/* Number of float32 network parameters (the length of `params`; for an
 * ensemble, the members' vectors one after the other). */
size_t nnp_param_count(const nnp_handle* h);

/* Replaces the network weights from a device vector in the `params` layout
 * (float32, nnp_param_count() entries; ensembles: all members, member-major);
 * enqueued on `stream`. */
nnp_status nnp_set_params_device(nnp_handle* h, const float* params_dev, void* stream);

/* Neighbor-list capacity per atom (default 128, range 16..512, rounded up to
 * a multiple of 16).  A larger capacity needs a larger workspace. */
nnp_status nnp_set_max_neighbors(nnp_handle* h, int32_t max_neighbors);

/* Box format of every later call on this handle (the paper's GFP example ran
 * in a periodic cell; Results, "Example: MLP for Anionic Green Fluorescent
 * Protein Chromophore in Water").  on == 0 (default): `box` is 3 floats,
 * the edges of an orthorhombic cell.  on != 0: `box` is 9 floats, the rows
 * a = (ax, 0, 0), b = (bx, by, 0), c = (cx, cy, cz) of a triclinic cell in
 * reduced form (ax, by, cz > 0; |bx|, |cx| <= ax/2; |cy| <= by/2).  The
 * image of a displacement is removed along c, then b, then a, each step
 * n = rint(fl32(d_k * fl32(1 / v_kk))), d -= fl32(v_k * n), float32 without
 * contraction; this is the minimum image when every perpendicular width is
 * at least twice the radial cutoff, which is required (else NNP_E_BOX, as is
 * a cell not in reduced form).  Atoms are binned in fractional coordinates. */
nnp_status nnp_set_triclinic(nnp_handle* h, int32_t on);

/* Force accumulation order of every later call on this handle.  Forces are
 * the negative energy gradient (Methods, "PyTorch Model Support"); how the
 * per-pair terms are summed is this library's choice.
 * on == 0 (default): each atom's adjoint adds its neighbors' terms with
 * floating-point atomics, so the last bits of a force depend on scheduling.
 * on != 0 (deterministic gather mode): one atom per wave in the symmetry-
 * function kernels; the adjoint writes each atom's dE_i/d(displacement) per
 * neighbor entry to the workspace (n_atoms x capacity x 16 more bytes, in
 * nnp_workspace_bytes), and a gather forms the force on atom a as the sum,
 * in a's neighbor-list order, of its own entries minus the matching entries
 * of its neighbors' lists.  Every energy and force is then a function of its
 * molecule alone: the same bits in any batch, any position, any run.  It is
 * slower and meant for debugging and reproducibility checks.  Graphs keep
 * the mode they were captured with.  NNP_E_INVALID for a null handle. */
nnp_status nnp_set_deterministic(nnp_handle* h, int32_t on);

/* Bytes of workspace an evaluation of this shape needs.  `box` is host memory
 * (3 floats) or NULL, as for nnp_energy_forces.  Returns 0 for invalid shapes. */
size_t nnp_workspace_bytes(const nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                           const float* box);

/* Energies and forces.
 *   n_atoms >= 0, n_mol >= 1 (n_mol == 1 when a box is given).
 *   pos         device, float32 [n_atoms][3], A.
 *   species     device, int32 [n_atoms], element index in [0, n_species).
 *   mol_offsets device, int32 [n_mol + 1]: molecule m owns atoms
 *               [mol_offsets[m], mol_offsets[m+1]); non-decreasing, first 0,
 *               last n_atoms.  There are no pairs across molecules.
 *   box         host, float32 [3] orthorhombic edge lengths (minimum image,
 *               every edge >= 2 * rc_rad, else NNP_E_BOX), or NULL.
 *   E           device, float64 [n_mol]: molecular energies (FP64 sums of the
 *               FP32 atomic energies and the self energies).
 *   F           device, float32 [n_atoms][3], or NULL for energy only.
 *   workspace   device, >= nnp_workspace_bytes(); caller-owned, not retained
 *               after the call's work completes.  Concurrent calls need
 *               distinct workspaces.
 * Allocates nothing; all work is enqueued on `stream`. */
nnp_status nnp_energy_forces(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                             const float* pos, const int32_t* species,
                             const int32_t* mol_offsets, const float* box,
                             double* E, float* F, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Energies and forces without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid allocation).  Arguments as nnp_energy_forces, plus
 *   status  device uint32 or NULL: receives the evaluation's device status
 *           word (the bits nnp_check() decodes) when the stream reaches the
 *           end of the call.
 * The workspace is a fixed 64 MiB device array inside the library (one per
 * device, held until the process ends); a system whose workspace would not
 * fit returns NNP_E_WORKSPACE and enqueues nothing.  At a neighbor capacity
 * of 128 that is about 3,000 atoms of seven elements with FP32 networks,
 * 6,000 with BF16, and 7,000 of four elements (BF16); the need is
 * nnp_workspace_bytes() less the weight-gradient partials it includes.  The call itself allocates nothing: no hipMalloc, no
 * event or stream creation.  Every call on a device uses the same array, so
 * calls that may overlap on one device (other streams, other threads) race
 * and must be serialised by the caller; consecutive calls on one stream are
 * safe.  Host-checkable errors return synchronously as for
 * nnp_energy_forces. */
nnp_status nnp_energy_forces_noalloc(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                                     const float* pos, const int32_t* species,
                                     const int32_t* mol_offsets, const float* box,
                                     double* E, float* F, uint32_t* status, void* stream);

/* A subset of a larger system (the ML/MM setting of Results, "Performance of
 * MLPs": the potential covers a 53-atom ligand inside a 134,099-atom system,
 * the rest is classical; mechanical embedding, so the potential sees only
 * the subset).  Subset atom i is row idx[i] of the full-system arrays:
 *   idx      device int32 [n_sub], distinct rows in [0, n_total);
 *   pos_all  device float32 [n_total][3];
 *   species, mol_offsets  device int32, per subset atom / subset molecule
 *            (subset-local, as in nnp_energy_forces);
 *   E        device float64 [n_mol], the subset's molecular energies;
 *   F_all    device float32 [n_total][3] or NULL: the subset's forces are
 *            ADDED to rows idx[i] (other rows untouched), so a caller can
 *            pass an array that already holds the classical forces.
 * Rows of idx outside [0, n_total) set NNP_E_INVALID in the status word and
 * are neither read nor written; repeated rows are the caller's error.  The
 * workspace is sized for n_sub atoms (nnp_workspace_bytes(h, n_sub, ...)). */
nnp_status nnp_energy_forces_subset(nnp_handle* h, int32_t n_sub, int32_t n_mol,
                                    const int32_t* idx, int32_t n_total, const float* pos_all,
                                    const int32_t* species, const int32_t* mol_offsets,
                                    const float* box, double* E, float* F_all, void* workspace,
                                    size_t ws_bytes, void* stream);

/* One spatial shard of a larger periodic system: the evaluation a GPU would
 * run in a slab (or brick) decomposition of one big box over several GPUs,
 * where each GPU owns the atoms of its region and holds copies ("ghosts")
 * of the atoms within the radial cutoff of its faces.  The paper's large
 * periodic simulations run one system over several GPUs (Results,
 * "Performance"); how a potential is split is this library's design.
 *   atoms [0, n_owned) are owned, [n_owned, n_atoms) ghosts; all interact
 *   (neighbor pairs ignore the split); positions in the full system's box;
 *   E  device float64 [2]: sum of E_i over the owned atoms, then over the
 *      ghosts (whose owners count them: a multi-GPU run adds up E[0] only);
 *   F  device float32 [n_atoms][3] = -dE[0]/dx for every atom: the owned
 *      atoms' forces from this shard's energy, and on the ghosts the parts
 *      that a run would send back to their owners and add there.
 * An owned atom's energy and force are exact when every atom within the
 * radial cutoff of it is present (owned or ghost); a ghost's own energy
 * needs no complete neighborhood since it is not counted.  box is required
 * (3 or 9 floats as set by nnp_set_triclinic).  Workspace:
 * nnp_workspace_bytes(h, n_atoms, 2, box).  NNP_E_INVALID for n_owned
 * outside [0, n_atoms], n_atoms < 1 or a null pointer. */
nnp_status nnp_energy_forces_owned(nnp_handle* h, int32_t n_atoms, int32_t n_owned,
                                   const float* pos, const int32_t* species, const float* box,
                                   double* E, float* F, void* workspace, size_t ws_bytes,
                                   void* stream);

/* Adjoint for L = sum_m dL_dE[m] * E_m.  Recomputes the forward pass (the
 * symmetry functions are recomputed, not stored between calls), then writes
 *   dL_dpos    device, float32 [n_atoms][3] = sum_m dL_dE[m] dE_m/dpos, or NULL;
 *   dL_dparams device, float32 [nnp_param_count()] in the `params` layout
 *              (overwritten, not accumulated), or NULL;
 *   E          device, float64 [n_mol], or NULL.
 * dL_dE is device float64 [n_mol].  Other arguments as nnp_energy_forces. */
nnp_status nnp_backward(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                        const float* pos, const int32_t* species,
                        const int32_t* mol_offsets, const float* box,
                        const double* dL_dE, float* dL_dpos, float* dL_dparams,
                        double* E, void* workspace, size_t workspace_bytes,
                        void* stream);

/* Waits for `stream`, then reads and clears the device status word of
 * `workspace`.  Returns NNP_OK or the first error bit set. */
nnp_status nnp_check(const nnp_handle* h, void* workspace, void* stream);

const char* nnp_status_string(nnp_status s);

/* Test and debug exports of intermediate results for the last evaluation run
 * in `workspace` (enqueued on `stream`):
 *   nnp_debug_neighbors: counts  device int32 [n_atoms][2] (radial, angular)
 *                        nbr     device int32 [n_atoms][max_neighbors]; row i
 *                        lists the angular neighbors first, then the rest.
 *   nnp_debug_aev:       runs staging, neighbor search and the symmetry
 *                        functions and writes G as float32 [n_atoms][F] in
 *                        input atom order into `aev` (device).
 *   nnp_debug_atom_energies: the atomic network outputs E_i (without self
 *                        energies) of the last nnp_energy_forces() or
 *                        nnp_backward() on `workspace` with the same n_atoms,
 *                        n_mol and box, float32 [n_models][n_atoms] in input
 *                        atom order, into `e_atom` (device). */
nnp_status nnp_debug_neighbors(nnp_handle* h, int32_t n_atoms, void* workspace,
                               size_t workspace_bytes, int32_t* counts,
                               int32_t* nbr, void* stream);
nnp_status nnp_debug_aev(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                         const float* pos, const int32_t* species,
                         const int32_t* mol_offsets, const float* box, float* aev,
                         void* workspace, size_t workspace_bytes, void* stream);
nnp_status nnp_debug_atom_energies(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                                   const float* box, void* workspace, size_t workspace_bytes,
                                   float* e_atom, void* stream);

/* Captured evaluations.  nnp_graph_capture() runs one nnp_energy_forces()
 * eagerly on `stream`, then captures the same call into a HIP graph; each
 * nnp_graph_launch() replays it.  The graph keeps the pointers it was
 * captured with: callers update the position (or species, offsets) buffers in
 * place between launches, with the same atom and molecule counts.  `stream`
 * must not be the legacy default stream (NULL).  The handle, workspace and
 * buffers must outlive the graph. */
typedef struct nnp_graph nnp_graph;
nnp_status nnp_graph_capture(nnp_handle* h, int32_t n_atoms, int32_t n_mol, const float* pos,
                             const int32_t* species, const int32_t* mol_offsets,
                             const float* box, double* E, float* F, void* workspace,
                             size_t workspace_bytes, void* stream, nnp_graph** out);
nnp_status nnp_graph_launch(nnp_graph* g, void* stream);
void nnp_graph_destroy(nnp_graph* g);

/* Per-stage device timing with HIP events, for benchmarks.  While enabled,
 * every evaluation records an event pair around each stage on its stream;
 * nnp_profile_collect() waits for the stream and adds the elapsed times to
 * per-stage totals.  Stage i is named by nnp_profile_stage_name(i) for
 * 0 <= i < nnp_profile_stage_count().  nnp_profile_read() copies the totals
 * (milliseconds) and launch counts; enabling resets them. */
nnp_status nnp_profile_enable(nnp_handle* h, int on);
nnp_status nnp_profile_collect(nnp_handle* h, void* stream);
int32_t nnp_profile_stage_count(void);
const char* nnp_profile_stage_name(int32_t i);
nnp_status nnp_profile_read(const nnp_handle* h, double* total_ms, int64_t* count, int32_t max);

/* ---------------------------------------------------------------------------
 * Molecular dynamics.  Velocity Verlet in eV, A, amu, fs with FP64 positions
 * and velocities and FP32 forces evaluated at the FP32 rounding of x:
 *   v += dt/2 * 9.648533e-3 * F / m;  x += dt * v;  F = F(x);
 *   v += dt/2 * 9.648533e-3 * F / m;
 * KE_m = 0.5 * sum m v^2 / 9.648533e-3 (eV, FP64).
 * ------------------------------------------------------------------------- */

/* n_steps velocity-Verlet steps of a packed batch, all on `stream`.
 *   x, v   device float64 [n_atoms][3], updated in place.
 *   F      device float32 [n_atoms][3]: on entry the forces at x (call
 *          nnp_energy_forces first), on exit the forces at the final x.
 *   mass   device float64 [n_atoms] (amu).
 *   E_pot, E_kin  device float64 [n_mol] at the final state (may be NULL).
 * The workspace must fit nnp_workspace_bytes() for this shape plus
 * 16 * n_atoms bytes. */
nnp_status nnp_md_steps(nnp_handle* h, int32_t n_atoms, int32_t n_mol,
                        double* x, double* v, float* F, const double* mass,
                        const int32_t* species, const int32_t* mol_offsets,
                        const float* box, double dt_fs, int32_t n_steps,
                        double* E_pot, double* E_kin, void* workspace,
                        size_t workspace_bytes, void* stream);

/* n_steps of LF-Middle Langevin dynamics (NVT; Methods, "Other Features":
 * the LF-Middle discretization; Results, GFP example: 300 K, 0.5 fs,
 * 1 / ps).  A leapfrog scheme whose velocities live at half steps.  From
 * x_n, v_{n-1/2} and F(x_n), each step does, per atom and component
 *   v += dt a;  x += dt/2 v;  v = c v + sqrt((1 - c^2) kB T / m) R;
 *   x += dt/2 v;  F = F(x)
 * with a = 9.648533e-3 F / m, c = exp(-friction * dt) and kB = 8.617333262e-5
 * eV/K.  R are standard normals: Philox4x32-10 (Salmon et al., SC '11) block
 * with counter (atom index, step mod 2^32, step div 2^32, 0) and key (seed
 * mod 2^32, seed div 2^32), words (0, 1) and (2, 3) through Box-Muller in
 * FP64 (u = (w + 1) 2^-32, theta = 2 pi w' 2^-32); the first three normals
 * drive x, y, z.  Step k of this call uses step index step0 + k, so a run
 * split over several calls draws the same numbers as one call.
 *   x, v   device float64 [n_atoms][3], in place (v: half-step velocities).
 *   F      device float32 [n_atoms][3]: forces at x on entry and on exit.
 *   mass   device float64 [n_atoms] (amu).
 *   temperature (K) >= 0, friction (1/ps) >= 0 (0 is leapfrog Verlet).
 *   E_pot  device float64 [n_mol] at the final x; E_kin of the final
 *          half-step velocities (either may be NULL).
 * Workspace as for nnp_md_steps.  NNP_E_INVALID for a negative temperature,
 * friction or step count, or dt <= 0. */
nnp_status nnp_langevin_steps(nnp_handle* h, int32_t n_atoms, int32_t n_mol, double* x,
                              double* v, float* F, const double* mass, const int32_t* species,
                              const int32_t* mol_offsets, const float* box, double dt,
                              int32_t n_steps, double temperature, double friction,
                              uint64_t seed, uint64_t step0, double* E_pot, double* E_kin,
                              void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of MD requests (molecules without a box).
 * A server owns fixed-capacity device buffers (max_atoms atoms, max_mols
 * molecules, sized within hbm_budget_bytes), a pending queue, and one
 * captured HIP graph of a whole velocity-Verlet step over the packed active
 * set.  Each nnp_server_step():
 *   1. hands over the results whose copies to the host have completed,
 *   2. drops requests that finished their steps and admits pending requests
 *      in arrival order while atoms, slots and the HBM budget allow (their
 *      x, v, species are copied to the device and the batch is repacked on
 *      the device),
 *   3. replays the step graph once over every active request,
 *   4. for requests whose last step that was, enqueues the copies of their
 *      state, energies and the device status word to pinned host memory
 *      behind an event, read by a later round: no round waits for the GPU
 *      (a round waits only when four rounds' results are still in flight, or
 *      when nothing is left to run).
 * Every request's trajectory is independent of the others in the batch.
 * Device errors (a neighbor list overflow, non-finite positions) are
 * reported per request by nnp_server_result: every request that was on the
 * device while a status bit was raised gets it.
 * ------------------------------------------------------------------------- */
nnp_status nnp_server_create(nnp_handle* h, size_t hbm_budget_bytes,
                             int32_t max_atoms, int32_t max_mols, double dt_fs,
                             const double* mass_amu /* host, [n_species] */,
                             void* stream, nnp_server** out);
/* The handle must outlive the server's calls; nnp_server_destroy does not
 * read it (it may run after nnp_destroy of the handle). */
void nnp_server_destroy(nnp_server* s);

/* Switches the server from velocity Verlet to LF-Middle Langevin dynamics
 * (NVT; Methods, "Other Features"; the scheme and the noise of
 * nnp_langevin_steps).  Only before the first nnp_server_step (else
 * NNP_E_INVALID).  A request's noise stream is keyed by its req_id (as the
 * seed) and counted by the atom's index inside the request and the request's
 * own step, so a request draws the same numbers alone and in any batch; its
 * submitted v is taken as v_{-1/2}, and its result holds x_n and v_{n-1/2}
 * after n steps (n + 1 force evaluations, as with velocity Verlet). */
nnp_status nnp_server_set_langevin(nnp_server* s, double temperature_K, double friction_per_ps);

/* Queues a request (host arrays are copied).  x, v: float64 [n_atoms][3];
 * species: int32 [n_atoms]; n_steps >= 1.  NNP_E_BUSY if the request can
 * never fit the server's capacity. */
nnp_status nnp_server_submit(nnp_server* s, int64_t req_id, int32_t n_atoms,
                             const double* x, const double* v,
                             const int32_t* species, int32_t n_steps);

/* One scheduling round (deliver, retire, admit, one MD step).  Returns after
 * the step has been enqueued; with no request left on the device it waits
 * for the results still in flight and delivers them. */
nnp_status nnp_server_step(nnp_server* s);

/* Requests admitted whose results have not been delivered yet (on the
 * device, or on their way back), and requests still queued. */
int32_t nnp_server_active(const nnp_server* s);
int32_t nnp_server_pending(const nnp_server* s);

/* Delivered request ids (up to `max`), oldest first; each id is reported
 * once.  Also delivers the results whose copies have completed (no wait). */
int32_t nnp_server_poll(nnp_server* s, int64_t* done_ids, int32_t max);

/* Result of a delivered request: final x, v (host float64 [n][3], may be
 * NULL), final potential and kinetic energy, and host wall-clock times
 * (seconds, steady clock) of submission, admission and delivery.  The
 * outputs are written in any case; the return value is the request's device
 * status (NNP_E_CAPACITY, NNP_E_NONFINITE, ... if a status bit was raised
 * while it was on the device, else NNP_OK). */
nnp_status nnp_server_result(nnp_server* s, int64_t req_id, double* x, double* v,
                             double* e_pot, double* e_kin, double* t_submit,
                             double* t_admit, double* t_done);

/* Server statistics into out[0 .. n): the atom and molecule capacity (after
 * fitting the HBM budget), atoms on the device now, the most atoms on the
 * device in one round, rounds run, rounds whose repack kept survivors and
 * admitted new requests, the most distinct request step counters in one
 * launch, and rounds that waited for a retire slot. */
nnp_status nnp_server_stats(const nnp_server* s, int64_t* out, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */

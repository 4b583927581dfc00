"""Parameter tables for the symmetry-function potential (inputs, not arithmetic).

The values follow the published ANI-2x conventions that the OpenMM 8 paper
benchmarks (Methods, "OpenMM-ML": ANI-1ccx with four elements, ANI-2x with
seven; "Optimization Through NNPOps": the ANI atom-centered symmetry
functions).  The paper prints none of these numbers; the choices below are
the workload definition and are recorded in the design notes:

* radial: cutoff 5.1 A, eta 19.7, 16 shifts evenly spaced on [0.8, 4.8875] A
  (both ends included), prefactor 0.25;
* angular: cutoff 3.5 A, eta 12.5, zeta 14.1, 4 radial shifts on [0.8, 2.6] A,
  8 angle shifts at the bin midpoints (2z+1)*pi/16, cosine scale 0.95;
* MLP widths 384-160-128-96-1 (four species) and 1008-256-192-160-1 (seven),
  CELU alpha 0.1; weights N(0, 1/fan_in), biases N(0, 0.1^2), output layer
  scaled by a force-scale factor; zero self energies.

All tables are float32: those float32 values are canonical for both the
oracle (which promotes them exactly to float64) and the GPU library.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

# ANI-2x element order (H, C, N, O, S, F, Cl); ANI-1ccx uses the first four.
SPECIES7 = ("H", "C", "N", "O", "S", "F", "Cl")
SPECIES4 = ("H", "C", "N", "O")

# Atomic masses in amu, in the element order above.
MASS_AMU = np.array([1.008, 12.011, 14.007, 15.999, 32.06, 18.998, 35.45],
                    dtype=np.float64)

# Output-layer scale that makes RMS |F| about 1 eV/A on the water boxes
# (four species: 1,500 waters; seven species: 7,667 waters).  With unit scale
# the FP64 reference gives RMS |F| = 0.194 and 0.168 eV/A; the scale is the
# rounded inverse (oracle/calibrate_force_scale.py recomputes it).
FORCE_SCALE = {4: 5.0, 7: 6.0}


@dataclass
class AEVTable:
    n_species: int
    rc_rad: np.float32
    eta_r: np.float32
    shf_r: np.ndarray  # float32 [n_r]
    rc_ang: np.float32
    eta_a: np.float32
    zeta: np.float32
    shf_a: np.ndarray  # float32 [n_a]
    shf_z: np.ndarray  # float32 [n_z]
    radial_prefactor: np.float32 = np.float32(0.25)
    angle_cos_scale: np.float32 = np.float32(0.95)

    @property
    def n_r(self) -> int:
        return int(self.shf_r.shape[0])

    @property
    def n_a(self) -> int:
        return int(self.shf_a.shape[0])

    @property
    def n_z(self) -> int:
        return int(self.shf_z.shape[0])


def feature_count(n_species: int, n_r: int = 16, n_a: int = 4, n_z: int = 8) -> int:
    """Length of one AEV row: radial blocks per species plus angular blocks per
    unordered species pair (the input width the first MLP layer is drawn for)."""
    return n_species * n_r + (n_species * (n_species + 1) // 2) * n_a * n_z


def aev_table(n_species: int, **overrides) -> AEVTable:
    f32 = np.float32
    t = AEVTable(
        n_species=n_species,
        rc_rad=f32(5.1),
        eta_r=f32(19.7),
        shf_r=np.linspace(0.8, 4.8875, 16).astype(np.float32),
        rc_ang=f32(3.5),
        eta_a=f32(12.5),
        zeta=f32(14.1),
        shf_a=np.linspace(0.8, 2.6, 4).astype(np.float32),
        shf_z=((2 * np.arange(8) + 1) * np.pi / 16).astype(np.float32),
    )
    for k, v in overrides.items():
        if isinstance(getattr(t, k), np.ndarray):
            v = np.asarray(v, dtype=np.float32)
        elif k != "n_species":
            v = f32(v)
        setattr(t, k, v)
    return t


@dataclass
class MLPTable:
    widths: tuple  # (F, h1, ..., 1)
    W: list  # W[s][l] float32 [out, in]
    b: list  # b[s][l] float32 [out]
    self_energy: np.ndarray  # float64 [S]
    celu_alpha: float = 0.1

    @property
    def n_species(self) -> int:
        return len(self.W)

    @property
    def n_layers(self) -> int:
        return len(self.widths) - 1

    def param_count(self) -> int:
        return sum(w.size + bb.size for ws, bs in zip(self.W, self.b) for w, bb in zip(ws, bs))

    def flat(self) -> np.ndarray:
        """All parameters as one float32 vector: species-major, then layer,
        then W (row-major out x in) followed by b."""
        parts = []
        for s in range(self.n_species):
            for l in range(self.n_layers):
                parts.append(self.W[s][l].ravel())
                parts.append(self.b[s][l].ravel())
        return np.concatenate(parts).astype(np.float32)

    def from_flat(self, v: np.ndarray) -> "MLPTable":
        v = np.asarray(v)
        W, b, o = [], [], 0
        for s in range(self.n_species):
            ws, bs = [], []
            for l in range(self.n_layers):
                n = self.W[s][l].size
                ws.append(v[o:o + n].reshape(self.W[s][l].shape)); o += n
                n = self.b[s][l].size
                bs.append(v[o:o + n].reshape(self.b[s][l].shape)); o += n
            W.append(ws); b.append(bs)
        return MLPTable(self.widths, W, b, self.self_energy.copy(), self.celu_alpha)

    def scaled_output(self, factor: float) -> "MLPTable":
        """The same networks with the output layer (W and b) times `factor`:
        energies and forces scale by it."""
        W = [[w.copy() for w in ws] for ws in self.W]
        b = [[x.copy() for x in bs] for bs in self.b]
        for s in range(self.n_species):
            W[s][-1] = (W[s][-1] * np.float32(factor)).astype(np.float32)
            b[s][-1] = (b[s][-1] * np.float32(factor)).astype(np.float32)
        return MLPTable(self.widths, W, b, self.self_energy.copy(), self.celu_alpha)


def default_widths(n_species: int) -> tuple:
    f = feature_count(n_species)
    return (f, 160, 128, 96, 1) if n_species == 4 else (f, 256, 192, 160, 1)


def mlp_table(n_species: int, seed: int | None = None, widths=None,
              out_scale: float | None = None) -> MLPTable:
    """Seeded Gaussian weights.  Draw order: species, then layer, W then b."""
    widths = tuple(widths or default_widths(n_species))
    if seed is None:
        seed = 100 + (0 if n_species == 4 else 1)
    if out_scale is None:
        out_scale = FORCE_SCALE.get(n_species, 1.0)
    rng = np.random.default_rng(seed)
    W, b = [], []
    n_layers = len(widths) - 1
    for _s in range(n_species):
        ws, bs = [], []
        for l in range(n_layers):
            fan_in, fan_out = widths[l], widths[l + 1]
            w = rng.standard_normal((fan_out, fan_in)) / np.sqrt(fan_in)
            bb = 0.1 * rng.standard_normal(fan_out)
            if l == n_layers - 1:
                w = w * out_scale
                bb = bb * out_scale
            ws.append(w.astype(np.float32))
            bs.append(bb.astype(np.float32))
        W.append(ws)
        b.append(bs)
    return MLPTable(widths, W, b, np.zeros(n_species, dtype=np.float64))

"""MI355X engine for ANI-style symmetry-function neural network potentials.

Python binding of the C ABI in include/nnp.h.  Every step of the energy,
force, gradient and MD path runs in the HIP library (libnnp.so); this module
only marshals torch device tensors (memory and streams) into pointers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import capi
from .capi import NNPError, NNP_MLP_BF16, NNP_MLP_FP32

__all__ = ["Potential", "NNPFunction", "Server", "Graph", "NNPError", "capi"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Potential:
    """A symmetry-function potential on the current GPU.

    Parameters are plain arrays: the radial/angular shift tables and scalars
    of the symmetry functions, the layer widths, and the flat float32
    parameter vector (per species, per layer: W row-major out x in, then b).
    A list of parameter vectors makes an ensemble of networks that share the
    widths and self energies; evaluations then return the ensemble mean.
    """

    def __init__(self, *, n_species, rc_rad, eta_r, shf_r, rc_ang, eta_a, zeta, shf_a, shf_z,
                 widths, params, celu_alpha=0.1, self_energy=None, radial_prefactor=0.25,
                 angle_cos_scale=0.95, precision="fp32", max_neighbors=128, triclinic=False,
                 deterministic=False):
        self._lib = capi.lib()
        self.n_species = int(n_species)
        self.widths = tuple(int(w) for w in widths)
        self.precision = precision
        self._keep = []
        shf_r = np.ascontiguousarray(shf_r, np.float32)
        shf_a = np.ascontiguousarray(shf_a, np.float32)
        shf_z = np.ascontiguousarray(shf_z, np.float32)
        self._keep += [shf_r, shf_a, shf_z]
        ap = capi.AevParams(self.n_species, float(rc_rad), float(eta_r), shf_r.size, _f32p(shf_r),
                            float(rc_ang), float(eta_a), float(zeta), shf_a.size, _f32p(shf_a),
                            shf_z.size, _f32p(shf_z), float(radial_prefactor),
                            float(angle_cos_scale))
        w = np.ascontiguousarray(self.widths, np.int32)
        members = list(params) if isinstance(params, (list, tuple)) else [params]
        ps = [np.ascontiguousarray(m, np.float32) for m in members]
        self.n_models = len(ps)
        es = None if self_energy is None else np.ascontiguousarray(self_energy, np.float64)
        self._keep += [w, es] + ps
        mps = (capi.MlpParams * len(ps))(*[
            capi.MlpParams(len(self.widths) - 1, w.ctypes.data_as(C.POINTER(C.c_int32)),
                           float(celu_alpha), _f32p(p),
                           None if es is None else es.ctypes.data_as(C.POINTER(C.c_double)))
            for p in ps])
        prec = NNP_MLP_BF16 if precision == "bf16" else NNP_MLP_FP32
        h = C.c_void_p()
        capi.check(self._lib.nnp_create_ensemble(C.byref(ap), mps, len(ps), prec, C.byref(h)),
                   "nnp_create_ensemble")
        self._h = h
        self.n_params = int(self._lib.nnp_param_count(h))
        if sum(p.size for p in ps) != self.n_params:
            raise ValueError(f"params have {sum(p.size for p in ps)} entries, "
                             f"expected {self.n_params}")
        if max_neighbors != 128:
            capi.check(self._lib.nnp_set_max_neighbors(h, int(max_neighbors)), "set_max_neighbors")
        self.max_neighbors = int(max_neighbors)
        # boxes: 3 edge lengths, or (triclinic) the 3 x 3 rows of a reduced cell
        self.triclinic = bool(triclinic)
        if self.triclinic:
            capi.check(self._lib.nnp_set_triclinic(h, 1), "set_triclinic")
        self._ws = None
        self.set_deterministic(deterministic)

    def set_deterministic(self, on: bool):
        """Deterministic gather mode for the forces (nnp_set_deterministic)."""
        self.deterministic = bool(on)
        capi.check(self._lib.nnp_set_deterministic(self._h, int(self.deterministic)),
                   "set_deterministic")

    @classmethod
    def from_tables(cls, aev, mlp, precision="fp32", **kw):
        """From objects with the attributes of ``workloads.AEVTable`` and
        ``workloads.MLPTable``."""
        return cls(n_species=aev.n_species, rc_rad=aev.rc_rad, eta_r=aev.eta_r, shf_r=aev.shf_r,
                   rc_ang=aev.rc_ang, eta_a=aev.eta_a, zeta=aev.zeta, shf_a=aev.shf_a,
                   shf_z=aev.shf_z, radial_prefactor=aev.radial_prefactor,
                   angle_cos_scale=aev.angle_cos_scale, widths=mlp.widths, params=mlp.flat(),
                   celu_alpha=mlp.celu_alpha, self_energy=mlp.self_energy, precision=precision,
                   **kw)

    @classmethod
    def ensemble_from_tables(cls, aev, mlps, precision="fp32", **kw):
        """An ensemble of networks (``workloads.MLPTable`` objects with equal
        widths) over one set of symmetry functions; self energies from the
        first member."""
        m0 = mlps[0]
        return cls(n_species=aev.n_species, rc_rad=aev.rc_rad, eta_r=aev.eta_r, shf_r=aev.shf_r,
                   rc_ang=aev.rc_ang, eta_a=aev.eta_a, zeta=aev.zeta, shf_a=aev.shf_a,
                   shf_z=aev.shf_z, radial_prefactor=aev.radial_prefactor,
                   angle_cos_scale=aev.angle_cos_scale, widths=m0.widths,
                   params=[m.flat() for m in mlps], celu_alpha=m0.celu_alpha,
                   self_energy=m0.self_energy, precision=precision, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self._lib.nnp_destroy(h)
            except Exception:
                pass
            self._h = None

    # ------------------------------------------------------------ workspace
    def _box_arg(self, box):
        if box is None:
            return None, None
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float32).reshape(9 if self.triclinic else 3))
        return b, C.c_void_p(b.ctypes.data)

    def workspace_bytes(self, n_atoms, n_mol, box=None):
        b, bp = self._box_arg(box)
        return int(self._lib.nnp_workspace_bytes(self._h, int(n_atoms), int(n_mol), bp))

    def workspace(self, n_atoms, n_mol, box=None, device=None):
        # an invalid shape or box sizes to 0: the library call then reports why
        need = max(self.workspace_bytes(n_atoms, n_mol, box), 256)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    def set_params(self, params: torch.Tensor):
        """Replace the network weights from a float32 device vector."""
        p = params.detach().to(torch.float32).contiguous()
        capi.check(self._lib.nnp_set_params_device(self._h, _ptr(p), _stream()), "set_params")

    # --------------------------------------------------------------- calls
    def energy_forces(self, pos, species, mol_offsets, box=None, forces=True, out=None):
        """E (float64 [n_mol]) and F (float32 [N, 3], or None)."""
        pos = pos.contiguous()
        n = pos.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        dev = pos.device
        E = torch.empty(n_mol, dtype=torch.float64, device=dev) if out is None else out[0]
        F = None
        if forces:
            F = torch.empty((n, 3), dtype=torch.float32, device=dev) if out is None else out[1]
        ws = self.workspace(n, n_mol, box, dev)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_energy_forces(
            self._h, n, n_mol, _ptr(pos), _ptr(species), _ptr(mol_offsets), bp, _ptr(E), _ptr(F),
            _ptr(ws), ws.numel(), _stream()), "nnp_energy_forces")
        return E, F

    def energy_forces_noalloc(self, pos, species, mol_offsets, box=None, forces=True, out=None):
        """As energy_forces, on the library's own fixed workspace (the call
        allocates no device memory).  Returns E, F and a device uint32 [1]
        holding the evaluation's status word."""
        pos = pos.contiguous()
        n = pos.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        dev = pos.device
        if out is None:
            E = torch.empty(n_mol, dtype=torch.float64, device=dev)
            F = torch.empty((n, 3), dtype=torch.float32, device=dev) if forces else None
            status = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            E, F, status = out
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_energy_forces_noalloc(
            self._h, n, n_mol, _ptr(pos), _ptr(species), _ptr(mol_offsets), bp, _ptr(E), _ptr(F),
            _ptr(status), _stream()), "nnp_energy_forces_noalloc")
        return E, F, status

    def energy_forces_subset(self, idx, pos_all, species, mol_offsets, F_all=None, box=None):
        """Energies of the subset rows idx of a larger system; its forces are
        added into F_all (float32 [n_total, 3]) when given.  Returns E."""
        idx = idx.to(torch.int32).contiguous()
        pos_all = pos_all.contiguous()
        n_sub = idx.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        E = torch.empty(n_mol, dtype=torch.float64, device=pos_all.device)
        ws = self.workspace(n_sub, n_mol, box, pos_all.device)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_energy_forces_subset(
            self._h, n_sub, n_mol, _ptr(idx), pos_all.shape[0], _ptr(pos_all), _ptr(species),
            _ptr(mol_offsets), bp, _ptr(E), _ptr(F_all), _ptr(ws), ws.numel(), _stream()),
            "nnp_energy_forces_subset")
        return E

    def energy_forces_owned(self, pos, species, n_owned, box):
        """One shard of a larger periodic system (nnp_energy_forces_owned):
        atoms [0, n_owned) owned, the rest ghosts.  Returns (E float64 [2]:
        owned and ghost energy sums, F float32 [N, 3] = -dE[0]/dpos)."""
        pos = pos.contiguous()
        n = pos.shape[0]
        E = torch.empty(2, dtype=torch.float64, device=pos.device)
        F = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
        ws = self.workspace(n, 2, box, pos.device)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_energy_forces_owned(
            self._h, n, int(n_owned), _ptr(pos), _ptr(species), bp, _ptr(E), _ptr(F), _ptr(ws),
            ws.numel(), _stream()), "nnp_energy_forces_owned")
        return E, F

    def backward(self, pos, species, mol_offsets, dL_dE, box=None, want_pos=True,
                 want_params=True):
        """(dL/dpos float32 [N,3] or None, dL/dparams float32 [P] or None, E)."""
        pos = pos.contiguous()
        n = pos.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        dev = pos.device
        dLdE = dL_dE.to(torch.float64).contiguous()
        gp = torch.empty((n, 3), dtype=torch.float32, device=dev) if want_pos else None
        gw = torch.empty(self.n_params, dtype=torch.float32, device=dev) if want_params else None
        E = torch.empty(n_mol, dtype=torch.float64, device=dev)
        ws = self.workspace(n, n_mol, box, dev)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_backward(
            self._h, n, n_mol, _ptr(pos), _ptr(species), _ptr(mol_offsets), bp, _ptr(dLdE),
            _ptr(gp), _ptr(gw), _ptr(E), _ptr(ws), ws.numel(), _stream()), "nnp_backward")
        return gp, gw, E

    def check(self):
        """Synchronise the current stream and raise on a device-side error."""
        if self._ws is None:
            return
        capi.check(self._lib.nnp_check(self._h, _ptr(self._ws), _stream()), "device status")

    def debug_neighbors(self, n_atoms):
        dev = self._ws.device
        counts = torch.empty((n_atoms, 2), dtype=torch.int32, device=dev)
        nbr = torch.empty((n_atoms, self.max_neighbors), dtype=torch.int32, device=dev)
        capi.check(self._lib.nnp_debug_neighbors(self._h, n_atoms, _ptr(self._ws),
                                                 self._ws.numel(), _ptr(counts), _ptr(nbr),
                                                 _stream()), "debug_neighbors")
        return counts, nbr

    def debug_atom_energies(self, n_atoms, n_mol, box=None):
        """Atomic network outputs E_i (no self energies) of the last
        evaluation, float32 [n_models, n_atoms] in input atom order."""
        dev = self._ws.device
        out = torch.empty((self.n_models, n_atoms), dtype=torch.float32, device=dev)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_debug_atom_energies(self._h, int(n_atoms), int(n_mol), bp,
                                                     _ptr(self._ws), self._ws.numel(), _ptr(out),
                                                     _stream()), "debug_atom_energies")
        return out

    def debug_aev(self, pos, species, mol_offsets, box=None):
        pos = pos.contiguous()
        n = pos.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        F = self.widths[0]
        out = torch.empty((n, F), dtype=torch.float32, device=pos.device)
        ws = self.workspace(n, n_mol, box, pos.device)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_debug_aev(self._h, n, n_mol, _ptr(pos), _ptr(species),
                                           _ptr(mol_offsets), bp, _ptr(out), _ptr(ws), ws.numel(),
                                           _stream()), "debug_aev")
        return out

    def capture(self, pos, species, mol_offsets, box=None, stream=None):
        """A replayable graph of energy_forces on these buffers (see
        nnp_graph_capture); returns a Graph whose .E and .F are the outputs.
        Update ``pos`` in place between launches."""
        return Graph(self, pos, species, mol_offsets, box, stream)

    # ---------------------------------------------------------- profiling
    def profile(self, on: bool):
        capi.check(self._lib.nnp_profile_enable(self._h, int(bool(on))), "profile_enable")

    def profile_collect(self):
        capi.check(self._lib.nnp_profile_collect(self._h, _stream()), "profile_collect")

    def profile_read(self):
        """{stage name: (total ms, launches)} since profiling was enabled."""
        n = int(self._lib.nnp_profile_stage_count())
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        capi.check(self._lib.nnp_profile_read(self._h, C.c_void_p(ms.ctypes.data),
                                              C.c_void_p(cnt.ctypes.data), n), "profile_read")
        return {self._lib.nnp_profile_stage_name(i).decode(): (float(ms[i]), int(cnt[i]))
                for i in range(n)}

    def md_steps(self, x, v, F, mass, species, mol_offsets, dt, n_steps, box=None):
        """Velocity-Verlet steps in place on float64 x, v (F: forces at x)."""
        n = x.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        Ep = torch.empty(n_mol, dtype=torch.float64, device=x.device)
        Ek = torch.empty(n_mol, dtype=torch.float64, device=x.device)
        ws = self.workspace(n, n_mol, box, x.device)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_md_steps(self._h, n, n_mol, _ptr(x), _ptr(v), _ptr(F),
                                          _ptr(mass), _ptr(species), _ptr(mol_offsets), bp,
                                          float(dt), int(n_steps), _ptr(Ep), _ptr(Ek), _ptr(ws),
                                          ws.numel(), _stream()), "nnp_md_steps")
        return Ep, Ek


    def langevin_steps(self, x, v, F, mass, species, mol_offsets, dt, n_steps, temperature,
                       friction, seed, step0=0, box=None):
        """LF-Middle Langevin steps in place on float64 x and half-step v
        (F: forces at x); friction in 1/ps.  Returns (E_pot, E_kin)."""
        n = x.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        Ep = torch.empty(n_mol, dtype=torch.float64, device=x.device)
        Ek = torch.empty(n_mol, dtype=torch.float64, device=x.device)
        ws = self.workspace(n, n_mol, box, x.device)
        b, bp = self._box_arg(box)
        capi.check(self._lib.nnp_langevin_steps(
            self._h, n, n_mol, _ptr(x), _ptr(v), _ptr(F), _ptr(mass), _ptr(species),
            _ptr(mol_offsets), bp, float(dt), int(n_steps), float(temperature), float(friction),
            int(seed), int(step0), _ptr(Ep), _ptr(Ek), _ptr(ws), ws.numel(), _stream()),
            "nnp_langevin_steps")
        return Ep, Ek


class Graph:
    """A captured energy + force evaluation (nnp_graph_*)."""

    def __init__(self, pot, pos, species, mol_offsets, box=None, stream=None):
        self.pot = pot
        self.stream = stream or torch.cuda.Stream()
        n = pos.shape[0]
        n_mol = mol_offsets.shape[0] - 1
        self.pos, self.species, self.off = pos, species, mol_offsets
        self.E = torch.empty(n_mol, dtype=torch.float64, device=pos.device)
        self.F = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
        self.ws = torch.empty(max(pot.workspace_bytes(n, n_mol, box), 256), dtype=torch.uint8,
                              device=pos.device)
        self._box, bp = pot._box_arg(box)
        g = C.c_void_p()
        torch.cuda.current_stream().synchronize()
        capi.check(pot._lib.nnp_graph_capture(
            pot._h, n, n_mol, _ptr(pos), _ptr(species), _ptr(mol_offsets), bp, _ptr(self.E),
            _ptr(self.F), _ptr(self.ws), self.ws.numel(), C.c_void_p(self.stream.cuda_stream),
            C.byref(g)), "nnp_graph_capture")
        self._g = g
        self.stream.synchronize()

    def launch(self):
        capi.check(self.pot._lib.nnp_graph_launch(self._g, C.c_void_p(self.stream.cuda_stream)),
                   "nnp_graph_launch")

    def synchronize(self):
        self.stream.synchronize()

    def check(self):
        capi.check(self.pot._lib.nnp_check(self.pot._h, _ptr(self.ws),
                                           C.c_void_p(self.stream.cuda_stream)), "device status")

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and g.value:
            try:
                self.pot._lib.nnp_graph_destroy(g)
            except Exception:
                pass
            self._g = None


class NNPFunction(torch.autograd.Function):
    """E = potential(pos, params) with a hand-written adjoint.

    forward(pos, params, potential, species, mol_offsets, box) -> E [n_mol].
    The backward recomputes the symmetry functions (nothing but the inputs is
    saved) and returns dL/dpos and dL/dparams from one library call.
    """

    @staticmethod
    def forward(ctx, pos, params, potential, species, mol_offsets, box=None):
        potential.set_params(params)
        E, _ = potential.energy_forces(pos.detach(), species, mol_offsets, box, forces=False)
        ctx.save_for_backward(pos, params)
        ctx.potential, ctx.species, ctx.off, ctx.box = potential, species, mol_offsets, box
        return E

    @staticmethod
    def backward(ctx, gE):
        pos, params = ctx.saved_tensors
        pot = ctx.potential
        pot.set_params(params)
        gp, gw, _ = pot.backward(pos.detach(), ctx.species, ctx.off, gE.detach(), ctx.box,
                                 want_pos=ctx.needs_input_grad[0],
                                 want_params=ctx.needs_input_grad[1])
        if gp is not None:
            gp = gp.to(pos.dtype)
        if gw is not None:
            gw = gw.to(params.dtype)
        return gp, gw, None, None, None, None


class Server:
    """Continuous-batching MD server (see nnp_server_* in include/nnp.h)."""

    def __init__(self, potential: Potential, hbm_budget_bytes: int, max_atoms: int, max_mols: int,
                 dt_fs: float, mass_amu):
        self._lib = potential._lib
        self.potential = potential
        m = np.ascontiguousarray(mass_amu, np.float64)
        s = C.c_void_p()
        capi.check(self._lib.nnp_server_create(potential._h, int(hbm_budget_bytes), int(max_atoms),
                                               int(max_mols), float(dt_fs),
                                               C.c_void_p(m.ctypes.data), _stream(), C.byref(s)),
                   "nnp_server_create")
        self._s = s

    def __del__(self):
        s = getattr(self, "_s", None)
        if s is not None and s.value:
            try:
                self._lib.nnp_server_destroy(s)
            except Exception:
                pass
            self._s = None

    def set_langevin(self, temperature_K, friction_per_ps):
        """LF-Middle Langevin instead of velocity Verlet (before the first step)."""
        capi.check(self._lib.nnp_server_set_langevin(self._s, float(temperature_K),
                                                     float(friction_per_ps)),
                   "nnp_server_set_langevin")

    def submit(self, req_id, x, v, species, n_steps):
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        sp = np.ascontiguousarray(species, np.int32)
        return self._lib.nnp_server_submit(self._s, int(req_id), int(sp.size),
                                           C.c_void_p(x.ctypes.data), C.c_void_p(v.ctypes.data),
                                           C.c_void_p(sp.ctypes.data), int(n_steps))

    def step(self):
        capi.check(self._lib.nnp_server_step(self._s), "nnp_server_step")

    @property
    def active(self):
        return int(self._lib.nnp_server_active(self._s))

    @property
    def pending(self):
        return int(self._lib.nnp_server_pending(self._s))

    def poll(self, max_n=1024):
        """Every delivered request id not reported before (the library hands
        them out max_n per call; this drains the queue)."""
        out = []
        ids = np.zeros(max_n, np.int64)
        while True:
            k = self._lib.nnp_server_poll(self._s, C.c_void_p(ids.ctypes.data), max_n)
            out += ids[:k].tolist()
            if k < max_n:
                return out

    def result(self, req_id, n_atoms, check=True):
        """Final state, energies and times of a delivered request.  With
        check, a device error raised while the request ran raises NNPError;
        otherwise the dict carries its status code."""
        x = np.zeros((n_atoms, 3))
        v = np.zeros((n_atoms, 3))
        vals = (C.c_double * 5)()
        code = self._lib.nnp_server_result(
            self._s, int(req_id), C.c_void_p(x.ctypes.data), C.c_void_p(v.ctypes.data),
            C.byref(vals, 0), C.byref(vals, 8), C.byref(vals, 16), C.byref(vals, 24),
            C.byref(vals, 32))
        if check:
            capi.check(code, "nnp_server_result")
        return dict(x=x, v=v, e_pot=vals[0], e_kin=vals[1], t_submit=vals[2], t_admit=vals[3],
                    t_done=vals[4], status=int(code))

    def stats(self):
        """Capacity and scheduling statistics (nnp_server_stats)."""
        out = np.zeros(8, np.int64)
        capi.check(self._lib.nnp_server_stats(self._s, C.c_void_p(out.ctypes.data), 8),
                   "nnp_server_stats")
        keys = ("capacity_atoms", "capacity_mols", "atoms_on_device", "peak_atoms", "rounds",
                "mixed_rounds", "max_phases_per_launch", "retire_waits")
        return dict(zip(keys, (int(x) for x in out)))

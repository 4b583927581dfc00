"""The allocation-free entry point (nnp_energy_forces_noalloc) against the
workspace entry point (nnp_energy_forces) on the same inputs, through the C
ABI: two calls in a row, the second on a smaller system, for both network
precisions, a periodic box, the size limit and the status word.

Bars: the two entry points run the same kernels, so energies agree to 1e-12
relative and forces to the FP32 parity bar (relative RMS <= 1e-5; only the
order of atomic force additions may differ).
"""
import numpy as np
import pytest
import torch

import workloads as w
from gpu_util import potential, to_dev, rel_rms

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def both(pot, s, box=None):
    pos, sp, off = to_dev(s)
    E1, F1 = pot.energy_forces(pos, sp, off, box)
    pot.check()
    E2, F2, st = pot.energy_forces_noalloc(pos, sp, off, box)
    torch.cuda.synchronize()
    return (E1.cpu().numpy(), F1.cpu().numpy(), E2.cpu().numpy(), F2.cpu().numpy(),
            int(st.cpu().item()))


def check_pair(E1, F1, E2, F2, st):
    assert st == 0
    assert np.all(np.isfinite(F2))
    assert np.max(np.abs(E2 - E1) / np.maximum(np.abs(E1), 1e-30)) <= 1e-12
    assert rel_rms(F2, F1) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_two_calls_second_smaller(prec):
    pot, _, _ = potential(7, prec)
    big = w.conformer_batch(40, 64, seed=1)           # 2,560 atoms in 40 molecules
    small = w.config_system(3, n_req=12)              # ragged molecules of 10-150 atoms
    assert small.n_atoms < big.n_atoms
    announce(f"noalloc {prec}: N={big.n_atoms}, then N={small.n_atoms}")
    r_big = both(pot, big)
    r_small = both(pot, small)
    check_pair(*r_big)
    check_pair(*r_small)
    # the small call again after the large one, the same numbers
    pos, sp, off = to_dev(small)
    E3, F3, st3 = pot.energy_forces_noalloc(pos, sp, off, None)
    torch.cuda.synchronize()
    assert int(st3.item()) == 0
    assert np.array_equal(E3.cpu().numpy(), r_small[2])


def test_noalloc_periodic_box():
    pot, _, _ = potential(4, "fp32")
    s = w.config_system(2)                             # 4,500 atoms, 35.5 A box
    announce(f"noalloc box: N={s.n_atoms}")
    check_pair(*both(pot, s, s.box))


def test_noalloc_rejects_oversize_and_reports_status():
    from paper_2310_03121_amd import NNPError
    pot, _, _ = potential(7, "bf16")
    s = w.conformer_batch(512, 64, seed=1)             # 32,768 atoms: beyond the fixed workspace
    pos, sp, off = to_dev(s)
    announce("noalloc: oversize rejected on the host")
    with pytest.raises(NNPError) as e:
        pot.energy_forces_noalloc(pos, sp, off, None)
    assert e.value.code == 8
    announce("noalloc: device status word of a bad species, then clean")
    s = w.config_system(3, n_req=4)
    pos, sp, off = to_dev(s)
    bad = sp.clone()
    bad[2] = 9
    _, _, st = pot.energy_forces_noalloc(pos, bad, off, None)
    torch.cuda.synchronize()
    assert int(st.item()) & 1
    _, F, st = pot.energy_forces_noalloc(pos, sp, off, None)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.all(np.isfinite(F.cpu().numpy()))

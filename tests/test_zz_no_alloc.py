"""The entry point that allocates nothing (mtp_energy_forces_stress_noalloc)
against mtp_energy_forces_stress, through the C ABI: two calls in a row on
the fixed scratch array, the second with a smaller input, in both forms, and
the rejection of an evaluation larger than the array."""
import numpy as np
import pytest
import torch

from paper_2304_13144_amd import api, synth
from tests.helpers import potential, theta_for

pytestmark = pytest.mark.gpu


def _case(reps):
    w = synth.workload2(reps=reps)
    pot = potential(w)
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta_for(2, pot))
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=64)
    return m, b, nb


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_allocating_entry_point(precision):
    big = _case((16, 16, 16))    # 16,384 atoms: the benchmark's configuration
    small = _case((5, 4, 3))     # 240 atoms, a ragged last block
    got = []
    for m, b, nb in (big, small):   # two calls in a row on the same scratch array
        got.append({k: v.cpu().numpy() for k, v in api.energy_forces_stress_noalloc(m, b, nb, precision).items()})
    torch.cuda.synchronize()
    for (m, b, nb), g in zip((big, small), got):
        want = {k: v.cpu().numpy() for k, v in api.energy_forces_stress(m, b, nb, precision).items()}
        for k in ("energy", "forces", "stress", "site_e"):
            assert g[k].shape == want[k].shape, k
            assert np.array_equal(g[k], want[k]), (precision, b.n_atoms, k, float(np.abs(g[k] - want[k]).max()))


def test_noalloc_rejects_evaluation_past_the_scratch():
    w = synth.workload2(reps=(16, 16, 16))
    m = api.Model.create(w.level, w.n_types, w.r_min, w.r_cut)
    m.set_params(theta_for(2, potential(w)))
    b = api.Batch(w.configs)
    nb = api.Neighbors().build(m, b, max_nbrs=256)   # pair gradients alone: 16,384 x 256 x 24 B = 96 MiB
    with pytest.raises(api.MtpError) as e:
        api.energy_forces_stress_noalloc(m, b, nb, "fp64")
    assert e.value.status == "MTP_E_CAPACITY"
    # the array is still usable afterwards
    small = _case((4, 4, 4))
    out = api.energy_forces_stress_noalloc(*small, "fp64")
    want = api.energy_forces_stress(*small, "fp64")
    assert torch.equal(out["forces"], want["forces"])

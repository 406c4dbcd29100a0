"""The paper's own example set-ups in lattice units.

Thread rupture (Sec. 3.1): a 336 x 8 x 8 gas region in a 360 x 40 x 40 box
breaks up under surface tension; the paper reports five bubbles at an
air-water surface tension and six at a four times smaller one.  The paper
gives neither the relaxation time nor the time step, so the lattice
mapping is a choice: tau = 0.55 (BGK) and sigma = 5e-3 and 1.25e-3 (the
4:1 ratio), FP64.  Its Ohnesorge numbers (0.11 and 0.22) are about seven times
the paper's (0.017 and 0.033): the mappings that match the paper's
(sigma ~ 0.02 at tau ~ 0.515) diverge within the first thousand steps in
this method, starting from the sharp corners of the region.  The counts
are qualitative only; parity unpinned.  Result: five bubbles in both cases
(the paper: five and six)."""
import numpy as np
import pytest

import scenes
from tests.parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_01632_amd as pkg
    pkg.lib()
    yield


def _rupture(sigma, steps=60000, every=1000):
    from paper_1604_01632_amd import Domain
    sc = scenes.gas_prism(tau=0.55, sigma=sigma)
    d = Domain.from_scene(sc, "fp64")
    m0 = d.read(())["scalars"]["total_mass"]
    counts = []
    for s in range(every, steps + 1, every):
        d.step(every)
        counts.append(len(d.bubbles()["id"]))
    s_ = d.read(())["scalars"]
    drift = abs(s_["total_mass"] - m0) / m0
    vols = np.sort(d.bubbles()["volume"])[::-1]
    d.close()
    return counts, drift, vols, s_["n_topology"]


@pytest.mark.timeout(600)
def test_thread_rupture_in_the_papers_geometry():
    out = {}
    for label, sigma in (("air-water", 5e-3), ("quarter", 1.25e-3)):
        counts, drift, vols, topo = _rupture(sigma)
        out[label] = counts
        say(f"[paper 3.1] sigma {sigma:g} ({label}): bubbles every 1000 steps "
            f"{counts}; final volumes {np.round(vols, 0).tolist()}; merges/splits {topo}; "
            f"mass drift {drift:.1e}")
        assert drift <= 1e-10
        assert counts[0] >= 1 and max(counts) >= 4  # the thread ruptured
    # the paper's five bubbles at the larger surface tension; at the smaller
    # one the paper reports six and this mapping gives five (four large
    # bubbles and one satellite of about 190 cells): the thread breaks at a
    # longer wavelength at the higher Ohnesorge number of the mapping
    assert out["air-water"][-1] == 5
    assert out["quarter"][-1] == 5

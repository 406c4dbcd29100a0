"""Debug knobs and failure detection of the C ABI: a fixed geometry
(freeze_conversions) against the oracle, and every device-side error forced
from host inputs (a non-finite PDF, a broken interface layer, a table too
small for a split, a drift bound below round-off); the watchdog never
changes what a step computes."""
import numpy as np
import pytest

import scenes
from scenes import GAS, IFACE, LIQ

from tests.parity import run_pair, say

pytestmark = pytest.mark.gpu

P0 = scenes.P0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    oracle.build(force=False)
    import paper_1604_01632_amd as pkg
    pkg.lib()
    yield


def _blobs():
    return scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=11,
                                                          sigma=1e-2))


def test_frozen_geometry_matches_oracle():
    """With conversions frozen the cell types and bubble IDs never change,
    and the flow, mass exchange and pressures still equal the oracle's bit
    for bit."""
    sc = _blobs()
    o, g = run_pair(sc, 40, 10, "frozen", freeze_conversions=1)
    assert np.array_equal(o.read()["cell_type"], sc.cell_type)
    assert np.array_equal(g.read(("cell_type",))["cell_type"], sc.cell_type)


def test_watchdog_leaves_results_unchanged():
    from paper_1604_01632_amd import Domain
    sc = _blobs()
    a = Domain.from_scene(sc, "fp32")
    b = Domain.from_scene(sc, "fp32", watchdog_every=7, watchdog_drift=1e-5)
    a.step(50)
    b.step(50)
    ra, rb = a.read(), b.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rb[key]), key


def _nan_scene(prec):
    from paper_1604_01632_amd import Domain
    sc = scenes.config("c1")
    N = sc.n
    o = Domain.from_scene(sc, prec)
    f = o.read(("f",))["f"]
    o.close()
    i = int(np.nonzero(sc.cell_type == LIQ)[0][100])
    f[3 * N + i] = np.nan
    return sc, f


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16dev"])
def test_nonfinite_pdf_reported(prec):
    """A NaN among the input PDFs of one liquid cell: the next synchronising
    call reports FSLBM_ENUMERIC (no watchdog needed: the stream-collide and
    interface kernels check every density they compute)."""
    from paper_1604_01632_amd import Domain, FslbmError, FSLBM_ENUMERIC
    sc, f = _nan_scene(prec)
    d = Domain(sc.params(precision={"fp64": 0, "fp32": 1, "fp16dev": 2}[prec]), sc.cell_type,
               sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles, f_init=f)
    d.step(3)
    with pytest.raises(FslbmError) as e:
        d.sync()
    assert e.value.code == FSLBM_ENUMERIC and "non-finite" in str(e.value)
    say(f"[watchdog] {prec}: {e.value}")


def _broken_layer_scene():
    """The static bubble with one interface cell turned liquid: a liquid
    cell next to gas (accepted only with the debug flag)."""
    sc = scenes.config("c1")
    N = sc.n
    nx = sc.nx
    t = sc.cell_type.copy()
    for i in np.nonzero(t == IFACE)[0]:
        x, y, z = i % nx, (i // nx) % sc.ny, i // (nx * sc.ny)
        if 0 < x < nx - 1 and t[i - 1] == GAS:
            t[i] = LIQ
            sc.phi[i] = 1.0
            sc.bubble_id[i] = -1
            return sc, t
    raise AssertionError("no interface cell next to gas along x")


def test_broken_interface_layer_detected():
    from paper_1604_01632_amd import (DEBUG_NO_LAYER_CHECK, Domain, FslbmError, FSLBM_EINVAL,
                                      FSLBM_ENUMERIC)
    sc, t = _broken_layer_scene()
    with pytest.raises(FslbmError) as e:
        Domain(sc.params(), t, sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles)
    assert e.value.code == FSLBM_EINVAL
    # accepted with the debug flag; without the watchdog nothing reports it
    quiet = Domain(sc.params(debug_flags=DEBUG_NO_LAYER_CHECK), t, sc.phi, sc.rho, sc.u,
                   sc.bubble_id, sc.bubbles)
    quiet.step(2)
    quiet.sync()
    d = Domain(sc.params(debug_flags=DEBUG_NO_LAYER_CHECK, watchdog_every=1), t, sc.phi, sc.rho,
               sc.u, sc.bubble_id, sc.bubbles)
    with pytest.raises(FslbmError) as e:
        d.step(3)
    assert e.value.code == FSLBM_ENUMERIC and "interface layer" in str(e.value)
    say(f"[watchdog] layer: {e.value}")


def test_table_full_on_split():
    """A filled neck splits one bubble into two: with room for one bubble
    the next synchronising call reports FSLBM_ECAPACITY."""
    from paper_1604_01632_amd import Domain, FslbmError, FSLBM_ECAPACITY
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)]
            + [(IFACE, 1.08, 0)] + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
            + [(LIQ, 1.0, -1)] * 3)
    sc = scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.05})
    ok = Domain.from_scene(sc, "fp64", max_bubbles=2)
    ok.step(4)
    assert len(ok.bubbles()["id"]) == 2
    d = Domain.from_scene(sc, "fp64", max_bubbles=1)
    d.step(4)
    with pytest.raises(FslbmError) as e:
        d.sync()
    assert e.value.code == FSLBM_ECAPACITY


def test_mass_drift_bound():
    """A drift bound below the FP32 round-off of the total mass fails the
    watchdog; a bound of 1e-6 passes."""
    from paper_1604_01632_amd import Domain, FslbmError, FSLBM_ENUMERIC
    sc = _blobs()
    good = Domain.from_scene(sc, "fp32", watchdog_every=5, watchdog_drift=1e-6)
    good.step(40)
    good.sync()
    bad = Domain.from_scene(sc, "fp32", watchdog_every=5, watchdog_drift=1e-300)
    with pytest.raises(FslbmError) as e:
        bad.step(40)
    assert e.value.code == FSLBM_ENUMERIC and "drifted" in str(e.value)


def test_batch_watchdog_names_the_member():
    from paper_1604_01632_amd import (Batch, DEBUG_NO_LAYER_CHECK, Domain, FslbmError,
                                      FSLBM_ENUMERIC)
    sc, t = _broken_layer_scene()
    good = Domain.from_scene(_blobs(), "fp32", watchdog_every=2)
    bad = Domain(sc.params(precision=1, debug_flags=DEBUG_NO_LAYER_CHECK, watchdog_every=2), t,
                 sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles)
    b = Batch([good, bad], tuning_cache_path="")
    with pytest.raises(FslbmError) as e:
        b.step(4)
    assert e.value.code == FSLBM_ENUMERIC and "batch member 1" in str(e.value)
    b.close()


def test_phase_mask_times_only_the_named_phases():
    from paper_1604_01632_amd import Domain, fslbm_get_timing, fslbm_set_timing
    d = Domain.from_scene(scenes.config("c1"), "fp32")
    fslbm_set_timing(d.handle, 2, ["bulk"])
    d.step(6)
    t = fslbm_get_timing(d.handle)
    assert t["steps"] == 3 and t["bulk_ms"] > 0
    assert t["iface_ms"] == 0 and t["label_ms"] == 0 and t["step_ms"] == t["bulk_ms"]


def test_copy_bandwidth_probe():
    import torch
    from paper_1604_01632_amd import fslbm_copy_bandwidth
    src = torch.arange(1 << 22, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    gbs = fslbm_copy_bandwidth(dst, src, 3)
    assert torch.equal(src, dst)
    assert 10.0 < gbs < 20000.0


def test_interface_list_capacity():
    """The per-slot arrays of the interface list hold iface_capacity cells:
    an initial state with more interface cells is refused, and a run whose
    interface grows past the capacity reports FSLBM_ECAPACITY (the list is
    cut, nothing is written beyond it)."""
    from paper_1604_01632_amd import Domain, FslbmError, FSLBM_ECAPACITY
    # an over-pressured bubble expands: its interface grows
    sc = scenes.spheres(n=(24, 24, 24), centers=((12.0, 12.0, 12.0),), radii=(5.0,),
                        p_init=(1.3 * P0,), rho_l=1.0, sigma=1e-3)
    n0 = int(np.count_nonzero(sc.cell_type == IFACE))
    with pytest.raises(FslbmError) as e:
        Domain.from_scene(sc, "fp32", iface_capacity=n0 - 1)
    assert e.value.code == FSLBM_ECAPACITY
    ref = Domain.from_scene(sc, "fp32")
    counts = []
    for _ in range(40):
        ref.step(1)
        counts.append(int(np.count_nonzero(ref.read(("cell_type",))["cell_type"] == IFACE)))
    # room for the start but not for the largest list of the run
    cap = max(n0, max(counts) - 1)
    assert max(counts) > cap >= n0
    d = Domain.from_scene(sc, "fp32", iface_capacity=cap)
    d.step(40)
    with pytest.raises(FslbmError) as e:
        d.sync()
    assert e.value.code == FSLBM_ECAPACITY and "interface list" in str(e.value)
    # with room for all of them the run is the default one
    ok = Domain.from_scene(sc, "fp32", iface_capacity=max(counts))
    ok.step(40)
    ra, rb = ok.read(), ref.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rb[key]), key

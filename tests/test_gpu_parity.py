"""GPU library (through the C ABI) against the CPU oracle, element by
element, on seeded synthetic scenes: FP64 form to 1e-12 with identical
cell types and bubble IDs."""
import numpy as np
import pytest

import scenes
from scenes import GAS, IFACE, LIQ
from tests.parity import compare_state, run_pair, say

pytestmark = pytest.mark.gpu

P0 = scenes.P0


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_01632_amd as pkg
    pkg.lib()  # fails loudly if the library is missing
    yield


def test_c1_static_bubble_fp64():
    """32^3 periodic box, one bubble R = 8, 200 steps (the plain-method
    configuration)."""
    run_pair(scenes.config("c1"), 200, 20, "c1")


@pytest.mark.parametrize("seed", [5, 3, 11])
def test_random_blobs_periodic(seed):
    """Several close bubbles with random pressures and a swirling flow:
    conversions every step, merges and splits within the horizon; ragged
    sizes that are not multiples of the wave size."""
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=seed,
                                                          sigma=1e-2))
    run_pair(sc, 80, 4, f"blobs-{seed}")


def test_random_blobs_walls_gravity_trt():
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(22, 19, 24), nblob=3, seed=7, walls=True,
                                                          sigma=5e-3, g=(0.0, 0.0, -2e-5)))
    run_pair(sc, 60, 5, "blobs-walls-trt", collision=1)


def test_merge_split_vanish_hand_cases():
    spec_merge = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, -0.08, 0)]
                  + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
                  + [(LIQ, 1.0, -1)] * 2)
    o, g = run_pair(scenes.layers(spec_merge, ny=4, nz=4, p_init={0: P0 * 1.1, 1: P0 * 0.9}), 4, 1,
                    "merge")
    assert o.bubbles()["id"].tolist() == [2]
    spec_split = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)]
                  + [(IFACE, 1.08, 0)] + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
                  + [(LIQ, 1.0, -1)] * 3)
    o, g = run_pair(scenes.layers(spec_split, ny=4, nz=4, p_init={0: P0 * 1.05}), 4, 1, "split")
    assert o.bubbles()["id"].tolist() == [1, 2]
    spec_vanish = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 1.1, 0)] + [(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 1)]
                   + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)] + [(LIQ, 1.0, -1)] * 2)
    o, g = run_pair(scenes.layers(spec_vanish, ny=3, nz=3), 3, 1, "vanish")
    assert o.bubbles()["id"].tolist() == [1]


@pytest.mark.parametrize("phi", [0.5, -0.05])
def test_lone_interface_rules(phi):
    """Interface cells that no longer separate liquid from gas: a lone layer
    inside the liquid fills (also below -eps), a single lone cell fills
    without turning its liquid neighbours, a liquid-free film empties; the
    bucket they feed is spread in the next steps."""
    lone = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, phi, 0)] + [(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 1)]
            + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)] + [(LIQ, 1.0, -1)] * 2)
    run_pair(scenes.layers(lone, ny=3, nz=3), 4, 1, f"lone-layer-{phi}")
    film = ([(LIQ, 1.0, -1)] * 2 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.4, 0)]
            + [(IFACE, 0.6, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)] + [(LIQ, 1.0, -1)] * 2)
    run_pair(scenes.layers(film, ny=3, nz=3), 4, 1, "film")
    spec = ([(LIQ, 1.0, -1)] * 8 + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=5, nz=5)
    i = 3 + len(spec) * (2 + 5 * 2)
    sc.cell_type[i] = IFACE
    sc.phi[i] = phi
    sc.bubble_id[i] = 0
    sc.bubbles.insert(0, (0, 0, -1.0, P0))
    run_pair(sc, 4, 1, f"lone-cell-{phi}")


def test_orifice_injection():
    sc = scenes.orifice(n=(16, 16, 20), r=3.0, g=1e-5, Q=0.05)
    run_pair(sc, 40, 10, "orifice")


def test_orifice_rim_capping():
    """An under-pressured inlet bubble pulls liquid over the orifice: the
    interface cells next to the inlet go over-full and are capped (they
    keep m = rho and pass the rest on) every step; bitwise against the
    oracle."""
    sc = scenes.orifice(n=(16, 16, 20), r=3.0, g=1e-5, Q=0.0)
    sc.bubbles = [(b[0], b[1], b[2], b[3] * 0.8) for b in sc.bubbles]
    nx, ny = sc.nx, sc.ny
    z = np.arange(sc.n) // (nx * ny)
    above = np.roll(sc.cell_type == scenes.INLET, nx * ny) & (z == 1)
    sc.phi = np.where(above, 0.999, sc.phi)
    o, g = run_pair(sc, 30, 5, "orifice-capping")
    d = o.read()
    assert np.any(d["phi"][above] == 1.0)  # capped cells in the final state


def test_flat_interface_and_all_liquid_edge_cases():
    """Degenerate scenes: a flat interface sliding in a periodic box, an
    all-liquid box, a one-cell-wide line and an all-gas box."""
    spec = [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)] + [(LIQ, 1.0, -1)] * 6 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3
    run_pair(scenes.layers(spec, ny=5, nz=4, velocity=(0.0, 0.04, -0.03), tau=0.7), 10, 5, "flat-slide")
    liq = scenes.spheres(n=(9, 7, 5), centers=(), radii=(), rho_l=1.0)
    run_pair(liq, 10, 5, "all-liquid")
    one = scenes.spheres(n=(1, 12, 1), centers=(), radii=(), rho_l=1.0)
    run_pair(one, 6, 3, "line")
    # no fluid at all: empty interface, candidate and new-cell lists, one
    # bubble made of gas cells only (total mass 0, bucket spread over no
    # interface cell)
    gas = scenes.layers([(GAS, 0.0, 0)] * 6, ny=5, nz=4)
    o, _ = run_pair(gas, 6, 3, "all-gas")
    assert o.bubbles()["volume"].tolist() == [120.0] and o.scalars()["total_mass"] == 0.0


def test_trigger_equals_labelling_every_step():
    """The topology trigger never misses an event: running with labelling
    forced every step gives bitwise the same state."""
    from paper_1604_01632_amd import Domain
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=5, sigma=1e-2))
    a = Domain.from_scene(sc, "fp64")
    b = Domain.from_scene(sc, "fp64", force_topology=1)
    for k in range(8):
        a.step(10)
        b.step(10)
        ra, rb = a.read(), b.read()
        for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
            assert np.array_equal(ra[key], rb[key]), (k, key)
        ba, bb = a.bubbles(), b.bubbles()
        for key in ba:
            assert np.array_equal(ba[key], bb[key]), (k, key)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_deterministic_and_restartable(precision):
    """The same run twice is bitwise equal; N steps straight equal N/2
    steps, a checkpoint through the boundary, a restore and N/2 steps."""
    from paper_1604_01632_amd import Domain
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(20, 18, 16), nblob=3, seed=3, sigma=1e-2))
    a = Domain.from_scene(sc, precision)
    b = Domain.from_scene(sc, precision)
    a.step(40)
    b.step(40)
    ra, rb = a.read(), b.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rb[key]), key
    c = Domain.from_scene(sc, precision)
    c.step(20)
    ck = c.read()
    bub = c.bubbles()
    params = sc.params(precision=1 if precision == "fp32" else 0)
    binit = [(int(i), int(f), float(v), 0.0) for i, f, v in zip(bub["id"], bub["flags"], bub["v_star"])]
    d = Domain(params, ck["cell_type"], ck["phi"], ck["rho"], ck["u"], ck["bubble_id"], binit,
               f_init=ck["f"], restore=ck["scalars"], mass_init=ck["mass"])
    d.step(20)
    rd = d.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rd[key]), key
    assert np.array_equal(a.bubbles()["v_star"], d.bubbles()["v_star"])


def test_fp32_and_fp16dev_accuracy_against_fp64_oracle():
    """Reduced-precision storage: same bubble count, volumes within 1e-3,
    total mass drift within 1e-6 on the static-bubble case."""
    import oracle
    from paper_1604_01632_amd import Domain
    sc = scenes.config("c1")
    o = oracle.Oracle.from_scene(sc)
    o.step(200)
    bo = o.bubbles()
    m0 = oracle.Oracle.from_scene(sc).scalars()["total_mass"]
    for prec, vtol in (("fp32", 1e-3), ("fp16dev", 1e-3)):
        g = Domain.from_scene(sc, prec)
        g.step(200)
        bg = g.bubbles()
        s = g.read(("cell_type",))["scalars"]
        say(f"[accuracy] c1 {prec}: V {bg['volume']} vs {bo['volume']}, mass drift "
            f"{abs(s['total_mass'] - m0) / m0:.2e}")
        assert bg["id"].tolist() == bo["id"].tolist()
        assert np.allclose(bg["volume"], bo["volume"], rtol=vtol)
        assert abs(s["total_mass"] - m0) <= 1e-6 * m0


def test_invalid_inputs_rejected():
    from paper_1604_01632_amd import Domain, FslbmError
    sc = scenes.config("c1")
    t = sc.cell_type.copy()
    g = np.nonzero(t == GAS)[0][0]
    # liquid next to gas breaks the closed interface layer
    nbr = g + 1
    t2 = t.copy()
    t2[nbr] = LIQ if t2[nbr] != GAS else t2[nbr]
    t2[g] = GAS
    i_liq = np.nonzero(t == LIQ)[0][0]
    t3 = t.copy()
    t3[i_liq] = GAS
    with pytest.raises(FslbmError):
        Domain(sc.params(), t3, sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles)
    with pytest.raises(FslbmError):
        Domain(sc.params(max_bubbles=0), t, sc.phi, sc.rho, sc.u, sc.bubble_id, sc.bubbles)
    bid = sc.bubble_id.copy()
    bid[g] = 77
    with pytest.raises(FslbmError):
        Domain(sc.params(), t, sc.phi, sc.rho, sc.u, bid, sc.bubbles)


def test_sampled_phase_timing_leaves_results_unchanged():
    """Event timing of every k-th step times exactly those steps, rejects a
    negative period, and does not change what the steps compute."""
    from paper_1604_01632_amd import Domain, FslbmError, fslbm_get_timing, fslbm_set_timing
    sc = scenes.config("c1")
    a = Domain.from_scene(sc, "fp32")
    b = Domain.from_scene(sc, "fp32")
    fslbm_set_timing(a.handle, 3)
    a.step(7)
    a.step(3)
    t = fslbm_get_timing(a.handle)
    assert t["steps"] == 4  # steps 0, 3, 6 and 9 of the ten
    assert t["bulk_ms"] > 0 and t["step_ms"] >= t["bulk_ms"]
    fslbm_set_timing(a.handle, 1)
    a.step(2)
    assert fslbm_get_timing(a.handle)["steps"] == 2
    fslbm_set_timing(a.handle, 0)
    a.step(1)
    assert fslbm_get_timing(a.handle)["steps"] == 0
    with pytest.raises(FslbmError):
        fslbm_set_timing(a.handle, -1)
    b.step(13)
    ra, rb = a.read(), b.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rb[key]), key


def test_fp32_step_with_walls_matches_oracle():
    """One FP32 step of a walled scene (gravity, TRT, blobs away from and
    next to the walls) from the state the GPU reached, run by the oracle
    from that same state: cell types, bubble IDs and the bubble table
    exact, the fields within FP32 rounding.  Covers the FP32 geometry that
    reads plain fill-level rows in the interior and mirrors samples at the
    walls."""
    import oracle
    from paper_1604_01632_amd import Domain
    from tests.parity import compare_fp32_step, near_tie, oracle_from_state
    oracle.build(force=False)
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(
        n=(26, 22, 20), nblob=5, seed=21, walls=True, g=(0.0, 0.0, -2e-4), rmin=3.0, rmax=5.0))
    params = sc.params(collision=1)
    g = Domain.from_scene(sc, "fp32", collision=1)
    g.step(25)
    before = g.read()
    bb, sb = g.bubbles(), before["scalars"]
    o = oracle_from_state(params, before, bb, sb)
    t_before = before["cell_type"].copy()
    _, normal = o.geometry()
    c = oracle.lattice()[0]

    def audit(i):
        return near_tie(i, t_before, normal, c, (sc.nz, sc.ny, sc.nx))
    audit.t_before = t_before
    o.step(1)
    g.step(1)
    dg = g.read()
    compare_fp32_step(o.read(), o.bubbles(), o.scalars(), dg, g.bubbles(), dg["scalars"],
                      sc.nx * sc.ny * sc.nz, params.get("eps_convert", 1e-2), audit)
    g.close()

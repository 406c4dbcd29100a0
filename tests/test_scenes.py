"""The seeded many-domain generators give valid inputs (the oracle's
creation checks: closed interface layer, one ID per touching gas region,
listed IDs) with the stated size and sphere distributions."""
import numpy as np

import scenes


def test_batch_domains_valid(oracle_lib):
    ds = scenes.batch_domains(count=24, seed=4)
    for sc in ds:
        assert {sc.nx, sc.ny, sc.nz} <= {32, 48, 64, 80, 96}
        assert 1 <= len(sc.bubbles) <= 8
    small = sorted(ds, key=lambda s: s.n)[:12]
    for sc in small:
        oracle_lib.Oracle.from_scene(sc)  # raises on invalid input


def test_serve_requests_valid(oracle_lib):
    reqs = scenes.serve_requests(count=64, seed=5)
    edges = np.array([r["edge"] for r in reqs])
    assert edges.min() >= 32 and edges.max() <= 192 and np.all(edges % 16 == 0)
    assert all(500 <= r["horizon"] <= 5000 for r in reqs)
    for r in sorted(reqs, key=lambda r: r["edge"])[:6]:
        oracle_lib.Oracle.from_scene(scenes.request_scene(r))


def test_pore_scene(oracle_lib):
    """The pore box (Sec. 3.2): valid input, the paper's proportions, an
    inlet bubble and an atmosphere at p0, hydrostatic liquid with p0 at the
    surface, and both lattice mappings consistent with their definitions."""
    sc = scenes.pore(r=4, theta=70.0, q_ml_min=1.0, tau=0.6, units=scenes.pore_units_similar(4))
    assert (sc.nx, sc.ny, sc.nz) == (30, 30, 60)
    flags = {b: f for b, f, _, _ in sc.bubbles}
    assert flags == {0: scenes.BUBBLE_INLET, 1: scenes.BUBBLE_ATMOSPHERE}
    assert sc.contact_angle == 70.0
    t = sc.cell_type.reshape(sc.nz, sc.ny, sc.nx)
    assert np.count_nonzero(t[0] == scenes.INLET) == np.count_nonzero(
        (np.add.outer((np.arange(30) + 0.5 - 15) ** 2, (np.arange(30) + 0.5 - 15) ** 2)) <= 16)
    assert np.all(t[-1] == scenes.WALL) and np.all(t[1:-1, :, 0] == scenes.WALL)
    o = oracle_lib.Oracle.from_scene(sc)  # raises on invalid input
    b = o.bubbles()
    assert b["pressure"][list(b["id"]).index(1)] == scenes.P0
    rho = sc.rho.reshape(sc.nz, sc.ny, sc.nx)
    zs = sc.meta["surface"]
    g = -sc.g[2]
    assert rho[5, 10, 10] == np.float64(1.0 + 3.0 * g * (zs - 5))
    # similarity mapping: Bond number and flow per capillary time of water-air
    u = scenes.pore_units_similar(10, sigma=0.002)
    assert u["g"] * 100 / u["sigma"] == np.float64(u["bond"])
    assert abs(u["bond"] - 998.12 * 9.81 * 1e-6 / 0.0728) < 1e-12
    # physical mapping: nu dt / dx^2 equals the lattice viscosity
    v = scenes.pore_units(30, 0.51)
    assert abs(1.002e-3 / 998.12 * v["dt"] / v["dx"] ** 2 - (0.51 - 0.5) / 3) < 1e-15
    assert abs(v["dx"] - 1e-3 / 30) < 1e-18

"""Pins of the bubble model (Sec. 2.3): labelling against scipy and brute
force, and hand-built merge (Sec. 2.3.1), split (Sec. 2.3.2) and vanish
cases whose outcome follows from the rules by hand."""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import scenes
from scenes import GAS, IFACE, LIQ

P0 = scenes.P0


def _scipy_label(mask3, periodic):
    """Components under 18-neighbour adjacency (structure of rank 3,
    connectivity 2), then joined across periodic faces; returned as the
    smallest flat index of each component."""
    st = ndimage.generate_binary_structure(3, 2)
    lab, n = ndimage.label(mask3, structure=st)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    nz, ny, nx = mask3.shape
    # join labels that touch across a periodic face: compare each cell with
    # its wrapped 18 neighbours
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        if not 1 <= abs(dx) + abs(dy) + abs(dz) <= 2:
            continue
        sh = lab
        ok = np.ones_like(mask3)
        for axis, d, per, n_ in ((2, dx, periodic[0], nx), (1, dy, periodic[1], ny), (0, dz, periodic[2], nz)):
            if d == 0:
                continue
            sh = np.roll(sh, -d, axis=axis)
            if not per:
                sl = [slice(None)] * 3
                sl[axis] = slice(-1, None) if d > 0 else slice(0, 1)
                ok = ok.copy()
                ok[tuple(sl)] = False
        both = (lab > 0) & (sh > 0) & ok
        for a, b in zip(lab[both].tolist(), sh[both].tolist()):
            ra, rb = find(a), find(b)
            if ra != rb:
                parent[max(ra, rb)] = min(ra, rb)
    flat = lab.ravel()
    out = np.full(flat.shape, -1, np.int64)
    roots = np.array([find(v) if v > 0 else 0 for v in flat])
    first = {}
    for i, r in enumerate(roots):
        if flat[i] > 0 and r not in first:
            first[r] = i
    for i, r in enumerate(roots):
        if flat[i] > 0:
            out[i] = first[r]
    return out


@pytest.mark.parametrize("seed", range(12))
def test_label_matches_scipy(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(3, 11, 3))  # nx, ny, nz
    per = tuple(int(v) for v in rng.integers(0, 2, 3))
    dens = rng.uniform(0.15, 0.5)
    m = rng.random(shape[::-1]) < dens
    got = oracle_lib.label(m.astype(np.uint8), shape, per)
    want = _scipy_label(m, per)
    assert np.array_equal(got, want)


def test_label_brute_force_tiny(oracle_lib):
    """All pairs of cells at 18-neighbour distance joined by repeated
    relaxation on random 4x4x4 masks (periodic and not)."""
    rng = np.random.default_rng(42)
    n = 4
    idx = np.arange(n ** 3)
    x, y, z = idx % n, (idx // n) % n, idx // (n * n)
    for trial in range(30):
        per = tuple(int(v) for v in rng.integers(0, 2, 3))
        m = rng.random(n ** 3) < rng.uniform(0.2, 0.6)
        lab = np.where(m, idx, -1)
        adj = []
        for i in range(n ** 3):
            for j in range(n ** 3):
                if i == j:
                    continue
                d = []
                ok = True
                for a, b, p in ((x[i], x[j], per[0]), (y[i], y[j], per[1]), (z[i], z[j], per[2])):
                    dd = abs(int(a) - int(b))
                    if p:
                        dd = min(dd, n - dd)
                    d.append(dd)
                if max(d) <= 1 and 1 <= sum(d) <= 2:
                    adj.append((i, j))
        changed = True
        while changed:
            changed = False
            for i, j in adj:
                if m[i] and m[j] and lab[j] < lab[i]:
                    lab[i] = lab[j]
                    changed = True
        got = oracle_lib.label(m.astype(np.uint8), (n, n, n), per)
        assert np.array_equal(got, lab)


def _run(oracle_lib, sc, steps=1):
    o = oracle_lib.Oracle.from_scene(sc)
    b0 = o.bubbles()
    o.step(steps)
    return o, b0, o.bubbles()


def test_merge_by_emptied_film(oracle_lib):
    """Two bubbles separated by one liquid layer; the interface layer of
    bubble 0 next to the film empties (phi < -eps), the film turns
    interface and touches bubble 1: one new bubble with V* = V*_0 + V*_1
    and V = V_0 + V_1 (Sec. 2.3.1) and a fresh ID."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, -0.08, 0)]
            + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.1, 1: P0 * 0.9})
    o, b0, b1 = _run(oracle_lib, sc)
    assert b0["id"].tolist() == [0, 1]
    assert b1["id"].tolist() == [2]
    assert o.scalars()["next_id"] == 3
    assert b1["v_star"][0] == pytest.approx(b0["v_star"].sum(), rel=1e-14)
    d = o.read()
    setc = np.isin(d["cell_type"], [GAS, IFACE])
    vol = np.sum(np.where(d["cell_type"][setc] == IFACE, 1 - d["phi"][setc], 1.0))
    assert b1["volume"][0] == pytest.approx(vol, rel=1e-13)
    assert b1["pressure"][0] == pytest.approx(P0 * b1["v_star"][0] / b1["volume"][0], rel=1e-14)
    assert np.all(d["bubble_id"][setc] == 2)


def test_split_by_filled_neck(oracle_lib):
    """A bubble whose two halves are joined only through one layer of
    nearly full interface cells; the layer fills (phi > 1 + eps) and turns
    liquid: two daughters with fresh IDs in order of their smallest cell
    index, each with the mother's pressure (Sec. 2.3.2), so that the gas
    amount p V is conserved."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)]
            + [(IFACE, 1.08, 0)] + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
            + [(LIQ, 1.0, -1)] * 3)
    sc = scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.05})
    o, b0, b1 = _run(oracle_lib, sc)
    d = o.read()
    assert b1["id"].tolist() == [1, 2]
    # daughter 1 holds the smaller cell indices (left half)
    left = d["bubble_id"].reshape(4, 4, -1)[0, 0, 4]
    right = d["bubble_id"].reshape(4, 4, -1)[0, 0, 10]
    assert (left, right) == (1, 2)
    # mother's pressure on the new state: p0 V*_old / V_old(new state)
    v_old = b1["volume"].sum()
    p_old = P0 * b0["v_star"][0] / v_old
    assert np.allclose(b1["pressure"], p_old, rtol=1e-14)
    assert b1["v_star"].sum() == pytest.approx(b0["v_star"][0], rel=1e-14)
    assert np.sum(b1["pressure"] * b1["volume"]) == pytest.approx(P0 * b0["v_star"][0], rel=1e-14)
    assert np.allclose(b1["v_star"] / b1["volume"], b0["v_star"][0] / v_old, rtol=1e-14)


def test_vanishing_bubble(oracle_lib):
    """A bubble made only of nearly full interface cells fills up and
    disappears; its gas amount leaves the table."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 1.1, 0)] + [(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 1)]
            + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)] + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=3, nz=3)
    o, b0, b1 = _run(oracle_lib, sc)
    assert b0["id"].tolist() == [0, 1]
    assert b1["id"].tolist() == [1]
    assert b1["v_star"][0] == b0["v_star"][1]


def test_unchanged_topology_keeps_ids(oracle_lib):
    sc = scenes.config("c1")
    o, b0, b1 = _run(oracle_lib, sc, steps=5)
    assert b1["id"].tolist() == [0]
    assert o.scalars()["n_topology"] == 0
    assert b1["v_star"][0] == b0["v_star"][0]


@pytest.mark.parametrize("phi", [0.5, -0.05])
def test_lone_interface_cell_fills(oracle_lib, phi):
    """An interface layer with liquid on both sides and no gas neighbour no
    longer separates liquid from gas: it is filled in the next step whatever
    its fill level (also below -eps, where filling wins over emptying and
    its liquid neighbours stay liquid), its bubble vanishes, and with no
    interface neighbour left its whole deficit m - rho = phi - 1 per cell
    goes to the bucket (fluid at rest in equilibrium: no mass exchange).
    The next step spreads the bucket evenly over the remaining interface
    cells and empties it."""
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, phi, 0)] + [(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 1)]
            + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)] + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=3, nz=3)
    m0 = oracle_lib.Oracle.from_scene(sc).scalars()["total_mass"]
    o, b0, b1 = _run(oracle_lib, sc)
    d = o.read()
    t = d["cell_type"].reshape(3, 3, -1)
    assert np.all(t[:, :, 2:5] == LIQ)
    assert b0["id"].tolist() == [0, 1]
    assert b1["id"].tolist() == [1]
    s = o.scalars()
    assert s["bucket"] == pytest.approx((phi - 1.0) * 9, rel=1e-13)
    assert s["total_mass"] == pytest.approx(m0, rel=1e-14)
    share = (phi - 1.0) * 9 / 18
    phi_before = d["phi"].reshape(3, 3, -1)[:, :, 7].copy()
    o.step(1)
    s = o.scalars()
    assert s["total_mass"] == pytest.approx(m0, rel=1e-14)
    if phi > 0:  # a share of -0.25 leaves the remaining cells interface
        assert s["bucket"] == 0.0
        d = o.read()
        assert np.all(d["cell_type"].reshape(3, 3, -1)[:, :, 7] == IFACE)
        assert np.allclose(d["phi"].reshape(3, 3, -1)[:, :, 7], phi_before + share, atol=1e-3)


def test_interface_film_without_liquid_empties(oracle_lib):
    """A two-cell interface film between two gas regions of one bubble has
    no liquid neighbour: it is emptied whatever its fill level (0.4, 0.6);
    no interface cell is left next to it, so its mass (phi rho, no exchange
    at rest) goes to the bucket; the bubble keeps its ID."""
    spec = ([(LIQ, 1.0, -1)] * 2 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.4, 0)]
            + [(IFACE, 0.6, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)] + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=3, nz=3)
    m0 = oracle_lib.Oracle.from_scene(sc).scalars()["total_mass"]
    o, b0, b1 = _run(oracle_lib, sc)
    d = o.read()
    t = d["cell_type"].reshape(3, 3, -1)
    assert np.all(t[:, :, 5] == GAS) and np.all(t[:, :, 6] == GAS)
    assert np.all(t[:, :, 2] == IFACE) and np.all(t[:, :, 9] == IFACE)
    assert b1["id"].tolist() == [0]
    s = o.scalars()
    assert s["bucket"] == pytest.approx((0.4 + 0.6) * 9, rel=1e-13)
    assert s["total_mass"] == pytest.approx(m0, rel=1e-14)


def test_single_lone_cell_below_threshold_fills(oracle_lib):
    """One interface cell inside the liquid, its own bubble, fill level
    below -eps: it has no gas neighbour, so it is filled (filling wins over
    emptying) and none of its liquid neighbours turns interface; its deficit
    phi - 1 goes to the bucket and its bubble vanishes."""
    spec = ([(LIQ, 1.0, -1)] * 8 + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 2 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=5, nz=5)
    nx = len(spec)
    i = 3 + nx * (2 + 5 * 2)
    sc.cell_type[i] = IFACE
    sc.phi[i] = -0.05
    sc.bubble_id[i] = 0
    sc.bubbles.insert(0, (0, 0, -1.0, P0))
    m0 = oracle_lib.Oracle.from_scene(sc).scalars()["total_mass"]
    o, b0, b1 = _run(oracle_lib, sc)
    d = o.read()
    t = d["cell_type"].reshape(5, 5, -1)
    assert np.all(t[:, :, :8] == LIQ)
    assert b0["id"].tolist() == [0, 1]
    assert b1["id"].tolist() == [1]
    s = o.scalars()
    assert s["bucket"] == pytest.approx(-1.05, rel=1e-13)
    assert s["total_mass"] == pytest.approx(m0, rel=1e-14)


def test_restart_from_saved_state_is_exact(oracle_lib):
    """A run continued from a saved state (fields, masses, bubble table,
    step, next ID, bucket) equals the uninterrupted run bit for bit, through
    conversions and topology changes; this is the path the full-size GPU
    checks use to hand a GPU state to the oracle."""
    import parity

    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(20, 18, 16), nblob=4, seed=5))
    params = sc.params()
    a = oracle_lib.Oracle.from_scene(sc)
    a.step(25)
    saved, sb, ss = a.read(), a.bubbles(), a.scalars()
    b = parity.oracle_from_state(params, saved, sb, ss)
    assert b.scalars()["total_mass"] == ss["total_mass"]
    t25 = ss["n_topology"]
    a.step(35)
    b.step(35)
    assert a.scalars()["n_topology"] > t25  # the continuation changed topology
    da, db = a.read(), b.read()
    fl = np.isin(da["cell_type"], [IFACE, LIQ])
    for k in ("cell_type", "bubble_id", "phi", "mass"):
        assert np.array_equal(da[k], db[k]), k
    N = sc.nx * sc.ny * sc.nz
    assert np.array_equal(da["f"].reshape(19, N)[:, fl], db["f"].reshape(19, N)[:, fl])
    ba, bb = a.bubbles(), b.bubbles()
    for k in ba:
        assert np.array_equal(ba[k], bb[k]), k
    sa, sb2 = a.scalars(), b.scalars()
    for k in ("step", "next_id", "bucket", "total_mass"):
        assert sa[k] == sb2[k], k

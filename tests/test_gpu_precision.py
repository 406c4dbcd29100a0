"""The reduced-precision forms (FP32 and FP16-deviation storage) against
the FP64 form over whole horizons: the thread-rupture workload (64x64x256,
20000 steps, several ruptures) and a detaching variant of the orifice
workload (bubbles pinch off, rise and coalesce).  The bar: the same bubble
count, volumes within 1e-3 relative with bubbles matched by position, and
total-mass drift at most 1e-6 relative.  The FP64 form reproduces the
oracle bit for bit on the parity cases; at these horizons it stands in for
the oracle, whose CPU run would take hours."""
import numpy as np
import pytest

import scenes
from tests.parity import centroids, match_by_centroid, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_01632_amd as pkg
    pkg.lib()
    yield


def _run(sc, prec, checkpoints):
    """Bubbles, their centroids and the mass drift at each checkpoint."""
    from paper_1604_01632_amd import Domain
    d = Domain.from_scene(sc, prec)
    m0 = d.read(())["scalars"]["total_mass"]
    out, done = {}, 0
    for c in checkpoints:
        while done < c:
            n = min(5000, c - done)
            d.step(n)
            d.sync()
            done += n
        r = d.read(("bubble_id",))
        b = d.bubbles()
        out[c] = dict(b=b, cent=centroids(r["bubble_id"], b["id"], (sc.nz, sc.ny, sc.nx)),
                      drift=abs(r["scalars"]["total_mass"] - m0) / m0,
                      topo=r["scalars"]["n_topology"])
    d.close()
    return out


def _compare(sc, name, checkpoints, min_bubbles):
    ref = _run(sc, "fp64", checkpoints)
    for prec in ("fp32", "fp16dev"):
        got = _run(sc, prec, checkpoints)
        for c in checkpoints:
            r, g = ref[c], got[c]
            nb = len(r["b"]["id"])
            assert nb >= min_bubbles.get(c, 1), (name, c, nb)
            assert len(g["b"]["id"]) == nb, (name, prec, c)
            m = match_by_centroid(r["cent"], g["cent"], (sc.nz, sc.ny, sc.nx))
            assert m is not None, (name, prec, c, "bubbles cannot be paired one to one")
            err = np.abs(g["b"]["volume"][m] - r["b"]["volume"]) / r["b"]["volume"]
            say(f"[precision] {name} {prec} step {c}: {nb} bubbles, max volume error "
                f"{err.max():.2e} (volumes {np.round(r['b']['volume'], 1).tolist()}), mass drift "
                f"{g['drift']:.2e} (fp64 {r['drift']:.1e}), merges/splits {g['topo']} "
                f"(fp64 {r['topo']})")
            assert err.max() <= 1e-3
            assert g["drift"] <= 1e-6


def test_reduced_precision_at_thread_rupture_horizon():
    """64x64x256 thread, 20000 steps: the thread ruptures into three
    bubbles in every form."""
    _compare(scenes.config("c2"), "c2", (20000,), {20000: 2})


def _perturbed(sc, eps, seed):
    """The scene with its interface fill levels moved by U(-eps, eps)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    it = sc.cell_type == scenes.IFACE
    sc.phi = np.where(it, sc.phi + rng.uniform(-eps, eps, sc.n), sc.phi)
    return sc


def test_reduced_precision_through_detachment():
    """The detaching orifice variant.  Before the first pinch-off (step
    2000, one growing bubble) the forms meet the full bar.  Through
    pinch-offs (steps 4000 and 7000: 2 and 3 bubbles in FP64) they keep the
    bubble count, the mass (drift <= 1e-6), the gas amount (sum of V*) and
    the total gas volume, but the volume of each daughter is fixed by the
    moment its neck closes, which is ill-conditioned: the FP64 run itself,
    with its initial fill levels moved by 1e-9 (below FP32 rounding), ends
    with daughter volumes several per cent apart.  Per bubble the reduced
    forms are therefore held to three times that FP64 spread, not to
    1e-3."""
    base = scenes.config("c3d")
    shape = (base.nz, base.ny, base.nx)
    cps = (2000, 4000, 7000)
    ref = _run(base, "fp64", cps)
    pert = _run(_perturbed(scenes.config("c3d"), 1e-9, 77), "fp64", cps)
    assert len(ref[2000]["b"]["id"]) == 1
    assert len(ref[4000]["b"]["id"]) == 2 and len(ref[7000]["b"]["id"]) == 3

    def per_bubble(r, g):
        m = match_by_centroid(r["cent"], g["cent"], shape)
        assert m is not None, "bubbles cannot be paired one to one"
        return np.abs(g["b"]["volume"][m] - r["b"]["volume"]) / r["b"]["volume"]

    spread = {c: per_bubble(ref[c], pert[c]) for c in cps}
    say(f"[precision] c3d fp64 perturbed by 1e-9: per-bubble volume spread "
        f"{ {c: np.round(v, 4).tolist() for c, v in spread.items()} }")
    for prec in ("fp32", "fp16dev"):
        got = _run(base, prec, cps)
        for c in cps:
            r, g = ref[c], got[c]
            assert len(g["b"]["id"]) == len(r["b"]["id"]), (prec, c)
            err = per_bubble(r, g)
            vs = abs(g["b"]["v_star"].sum() - r["b"]["v_star"].sum()) / r["b"]["v_star"].sum()
            vt = abs(g["b"]["volume"].sum() - r["b"]["volume"].sum()) / r["b"]["volume"].sum()
            say(f"[precision] c3d {prec} step {c}: {len(r['b']['id'])} bubbles, per-bubble volume "
                f"error {np.round(err, 4).tolist()} (fp64 under 1e-9: "
                f"{np.round(spread[c], 4).tolist()}), total volume {vt:.1e}, sum V* {vs:.1e}, "
                f"mass drift {g['drift']:.1e}")
            assert g["drift"] <= 1e-6
            assert vs <= 1e-9
            assert vt <= 5e-3
            if c == 2000:
                assert err.max() <= 1e-3
            else:
                assert err.max() <= max(1e-3, 3 * spread[c].max())

"""The paper's split trigger (Sec. 2.3.2: anti-parallel normals of two
interface sections of one bubble next to a liquid cell) as an option beside
the exact trigger.  Labelling decides nothing by itself: a run that finds
no topology change keeps every ID, so a trigger that fires on every real
split gives bitwise the results of labelling every step (the oracle's
rule).  These tests run the normals trigger against labelling on every
step and count the splits it misses: steps after which one bubble ID
covers more than one connected gas region."""
import numpy as np
import pytest

import scenes

from tests.parity import say

pytestmark = pytest.mark.gpu

KEYS = ("cell_type", "bubble_id", "phi", "mass", "f")


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


def pending_splits(state, shape, periodic) -> int:
    """Bubble IDs whose cells form more than one connected component of the
    gas region (18-neighbour adjacency): splits not yet detected."""
    import oracle
    t = state["cell_type"]
    inset = (t == scenes.GAS) | (t == scenes.IFACE) | (t == scenes.INLET)
    lab = oracle.label(inset.astype(np.uint8), shape, periodic)
    ids = state["bubble_id"][inset]
    comps = lab[inset]
    n = 0
    for b in np.unique(ids):
        if len(np.unique(comps[ids == b])) > 1:
            n += 1
    return n


def _walk(sc, steps, prec="fp64", start=0, every=1):
    """Step a normals-trigger domain and a domain labelled every step side
    by side; returns (missed-split steps, first step whose states differ,
    label runs of each)."""
    from paper_1604_01632_amd import Domain, TRIGGER_NORMALS
    a = Domain.from_scene(sc, prec, split_trigger=TRIGGER_NORMALS, trigger_cos=-0.5)
    b = Domain.from_scene(sc, prec, force_topology=1)
    e = Domain.from_scene(sc, prec)  # the exact trigger, for its firing count
    if start:
        a.step(start)
        b.step(start)
        e.step(start)
    shape = (sc.nx, sc.ny, sc.nz)
    missed, first_diff = 0, None
    for s in range(start + every, start + steps + 1, every):
        a.step(every)
        b.step(every)
        e.step(every)
        ra = a.read(("cell_type", "bubble_id"))
        p = pending_splits(ra, shape, sc.periodic)
        missed += p > 0
        if first_diff is None:
            rb = b.read(("cell_type", "bubble_id"))
            if not (np.array_equal(ra["cell_type"], rb["cell_type"])
                    and np.array_equal(ra["bubble_id"], rb["bubble_id"])):
                first_diff = s
    sa, sb = a.read(())["scalars"], b.read(())["scalars"]
    full_equal = all(np.array_equal(x, y) for x, y in zip(
        (a.read(KEYS)[k] for k in KEYS), (b.read(KEYS)[k] for k in KEYS)))
    return dict(missed_steps=missed, first_diff=first_diff, runs_normals=sa["n_label_runs"],
                runs_exact=e.read(())["scalars"]["n_label_runs"],
                runs_every_step=sb["n_label_runs"], topology=sb["n_topology"],
                bubbles=(len(a.bubbles()["id"]), len(b.bubbles()["id"])), equal=full_equal)


@pytest.mark.parametrize("seed", [11, 3, 5])
def test_normals_trigger_on_blobs(seed):
    """Random blobs with merges and splits: the normals trigger against
    labelling every step.  Merges are found exactly by both; a split the
    normals trigger misses shows up as a bubble spanning two regions."""
    sc = scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=seed,
                                                          sigma=1e-2))
    r = _walk(sc, 80)
    say(f"[trigger] blobs-{seed}: {r}")
    assert r["runs_normals"] <= r["runs_every_step"]
    # every state that differs from labelling every step is explained by a
    # missed split
    if r["first_diff"] is not None:
        assert r["missed_steps"] > 0
    else:
        assert r["equal"]


def test_normals_trigger_through_first_thread_rupture():
    """The 64x64x256 thread (the thread-rupture workload) from step 1250
    through its first ruptures: the paper's trigger against labelling
    every step, FP64."""
    sc = scenes.config("c2")
    r = _walk(sc, 250, start=1250, every=2)
    say(f"[trigger] c2 steps 1252-1500: {r}")
    assert r["topology"] >= 1  # the thread ruptured in the window
    assert r["runs_normals"] < r["runs_every_step"]
    if r["first_diff"] is not None:
        assert r["missed_steps"] > 0


def test_normals_trigger_in_the_256_rupture_window():
    """The 256^3 thread lattice (FP32) through its rupture epoch: after every
    step of 1121-1220 the gas region is flooded on the host.  The exact
    trigger never leaves a split pending; the normals trigger may detect a
    split late, and both end with the same number of bubbles."""
    import torch
    from paper_1604_01632_amd import Domain, TRIGGER_NORMALS
    sc = scenes.config("p1")
    shape = (sc.nx, sc.ny, sc.nz)
    out = {}
    for name, over in (("normals", dict(split_trigger=TRIGGER_NORMALS, trigger_cos=-0.5)),
                       ("exact", {})):
        d = Domain.from_scene(sc, "fp32", **over)
        d.step(1120)
        pending = []
        for s in range(1121, 1221):
            d.step(1)
            p = pending_splits(d.read(("cell_type", "bubble_id")), shape, sc.periodic)
            if p:
                pending.append((s, p))
        s_ = d.read(())["scalars"]
        out[name] = dict(pending=pending, label_runs=s_["n_label_runs"],
                         topology=s_["n_topology"], bubbles=len(d.bubbles()["id"]))
        say(f"[trigger] p1 {name}: {out[name]}")
        d.close()
        del d
        torch.cuda.empty_cache()
    assert out["exact"]["pending"] == []
    assert out["exact"]["topology"] >= 40
    assert out["normals"]["bubbles"] == out["exact"]["bubbles"]
    assert out["normals"]["label_runs"] < out["exact"]["label_runs"]

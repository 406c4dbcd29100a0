"""Batched form through the C ABI: many domains of uneven sizes advanced by
one graph launch per step compute exactly what each domain computes alone
(bit for bit), across repeated graph replays with host reads between them,
odd step counts and a member stepped on its own; the FP64 batch matches the
oracle; the autotuning choice is cached."""
import numpy as np
import pytest

import scenes
from tests.parity import compare_state, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_01632_amd as pkg
    pkg.lib()
    yield


def _scenes():
    return [
        scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=5, sigma=1e-2)),
        scenes.merge_ids_if_touching(scenes.random_blobs(n=(22, 19, 24), nblob=3, seed=7, walls=True,
                                                         sigma=5e-3, g=(0.0, 0.0, -2e-5))),
        scenes.config("c1"),
        scenes.merge_ids_if_touching(scenes.random_blobs(n=(16, 20, 18), nblob=3, seed=3, sigma=1e-2)),
        scenes.orifice(n=(16, 16, 20), r=3.0, g=1e-5, Q=0.05),
        # wetting at 70 degrees and an atmosphere at the top
        scenes.pore(r=3, n=(20, 20, 32), tau=0.6, top_gas=5, theta=70.0, q_ml_min=1.0,
                    units=dict(g=2e-4, sigma=2e-3, q_per_ml_min=0.05)),
        scenes.batch_domains(count=1, seed=11, extents=(32, 48))[0],
    ]


def _same(a, b, label):
    ra, rb = a.read(), b.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rb[key]), f"{label}: {key}"
    assert ra["scalars"] == rb["scalars"], label
    ba, bb = a.bubbles(), b.bubbles()
    for key in ba:
        assert np.array_equal(ba[key], bb[key]), f"{label}: bubble {key}"


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_batch_equals_each_domain_alone(precision, tmp_path):
    from paper_1604_01632_amd import Batch, Domain

    scs = _scenes()
    over = [dict(collision=1) if k == 1 else {} for k in range(len(scs))]
    alone = [Domain.from_scene(sc, precision, **o) for sc, o in zip(scs, over)]
    mixed = [Domain.from_scene(sc, precision, **o) for sc, o in zip(scs, over)]
    b = Batch(mixed, tuning_cache_path=tmp_path / "tune.txt")
    info = b.info()
    say(f"[batch] {precision}: tuned {info}")
    assert info["bulk_threads"] in (128, 256) and info["from_cache"] == 0
    assert info["order"] in (0, 1, 2) and info["list_cells"] in (1024, 2048, 4096)
    assert all(t > 0 for t in info["probe_ms"])  # nine probes
    done = 0
    for n in (1, 1, 3, 5, 2):
        for d in alone:
            d.step(n)
        b.step(n)
        done += n
        for k, (a, m) in enumerate(zip(alone, mixed)):
            _same(a, m, f"{precision} domain {k} after {done} steps")
    # a member stepped on its own shifts its parity; the batch follows
    alone[2].step(1)
    mixed[2].step(1)
    for d in alone:
        d.step(4)
    b.step(4)
    for k, (a, m) in enumerate(zip(alone, mixed)):
        _same(a, m, f"{precision} domain {k} after the parity shift")
    b.close()
    b2 = Batch(mixed, tuning_cache_path=tmp_path / "tune.txt")
    i2 = b2.info()
    assert i2["from_cache"] == 1
    assert (i2["bulk_threads"], i2["order"], i2["list_cells"]) == (
        info["bulk_threads"], info["order"], info["list_cells"])
    assert b2.info()["bulk_threads"] == info["bulk_threads"]
    b2.close()


def test_batch_fp64_matches_oracle():
    import oracle
    from paper_1604_01632_amd import Batch, Domain

    scs = _scenes()[:6]
    doms = [Domain.from_scene(sc, "fp64") for sc in scs]
    orcs = [oracle.Oracle.from_scene(sc) for sc in scs]
    b = Batch(doms)
    for _ in range(3):
        b.step(7)
        for k, (o, d) in enumerate(zip(orcs, doms)):
            o.step(7)
            compare_state(o, d, f"batch domain {k}")
    b.close()


def test_batch_rejects_bad_input():
    from paper_1604_01632_amd import Batch, Domain, FslbmError

    sc = scenes.config("c1")
    a = Domain.from_scene(sc, "fp64")
    c = Domain.from_scene(sc, "fp32")
    with pytest.raises(FslbmError):
        Batch([a, c])
    with pytest.raises(FslbmError):
        Batch([a, a])


@pytest.mark.parametrize("case", ["thread_64x64x256", "orifice_48x48x96"])
def test_larger_domain_alone_equals_batch_of_one(case):
    """A domain stepped on its own and the same domain in a batch of one
    (graph launches of the batched kernels) give the same state bit for
    bit over many steps of a larger scene, checked twice along the way:
    a thread rupture with its conversions and labelling runs, and a walled,
    non-periodic box with an inlet."""
    from paper_1604_01632_amd import Batch, Domain

    if case.startswith("thread"):
        sc, steps = scenes.config("c2"), (700, 800)
    else:
        sc, steps = scenes.orifice(n=(48, 48, 96), r=5.0, g=1e-5, Q=0.05), (300, 300)
    alone = Domain.from_scene(sc, "fp32")
    other = Domain.from_scene(sc, "fp32")
    b = Batch([other], tuning_cache_path="")
    done = 0
    for n in steps:
        alone.step(n)
        b.step(n)
        done += n
        say(f"[alone-vs-batch] {case}: {done} steps, bubbles {len(alone.bubbles()['id'])}")
        _same(alone, other, f"{case} after {done} steps")
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_reset_members_come_and_go(precision):
    """A batch whose members change (fslbm_batch_reset: a serving loop's
    admissions and completions) keeps computing what each domain computes
    alone, bit for bit: members leave, join, rejoin with another parity."""
    from paper_1604_01632_amd import Batch, Domain

    scs = _scenes()[:4]
    alone = [Domain.from_scene(sc, precision) for sc in scs]
    mixed = [Domain.from_scene(sc, precision) for sc in scs]
    steps = [0] * len(scs)
    b = Batch(mixed[:2], tuning_cache_path="", capacity=len(scs))

    def run(members, n):
        b.step(n)
        for k in members:
            steps[k] += n

    run([0, 1], 7)
    b.reset([mixed[1], mixed[2]])
    run([1, 2], 4)
    mixed[3].step(3)  # stepped alone before it joins: another parity
    steps[3] += 3
    b.reset([mixed[3], mixed[0], mixed[1], mixed[2]])
    run([3, 0, 1, 2], 5)
    b.reset([mixed[2]])
    run([2], 2)
    with pytest.raises(Exception):
        b.reset(mixed + [Domain.from_scene(scs[0], precision)])  # beyond the capacity
    b.close()
    for k, (a, m) in enumerate(zip(alone, mixed)):
        a.step(steps[k])
        _same(a, m, f"reset member {k} after {steps[k]} steps")

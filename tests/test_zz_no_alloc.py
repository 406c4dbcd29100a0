"""The batched form with its tables in the library's static device array
(fslbm_batch_create_noalloc, for callers that cannot allocate) computes bit
for bit what the batched form with a caller workspace computes: two calls
in a row, the second on a smaller input."""
import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu

KEYS = ("cell_type", "bubble_id", "phi", "mass", "f")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_01632_amd as pkg
    pkg.lib()
    yield


def _scenes(big: bool):
    if big:
        return [
            scenes.merge_ids_if_touching(scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=11,
                                                             sigma=1e-2)),
            scenes.merge_ids_if_touching(scenes.random_blobs(n=(22, 19, 24), nblob=3, seed=7,
                                                             walls=True, sigma=5e-3,
                                                             g=(0.0, 0.0, -2e-5))),
            scenes.orifice(n=(16, 16, 20), r=3.0, g=1e-5, Q=0.05),
        ]
    return [
        scenes.merge_ids_if_touching(scenes.random_blobs(n=(16, 14, 12), nblob=2, seed=3,
                                                         sigma=1e-2)),
        scenes.orifice(n=(12, 12, 16), r=2.5, g=1e-5, Q=0.05),
    ]


def _run(scs, noalloc: bool, prec: str):
    import paper_1604_01632_amd as F
    doms = [F.Domain.from_scene(sc, prec) for sc in scs]
    if noalloc:
        h = F.fslbm_batch_create_noalloc([d.handle for d in doms])
        step = lambda n: F.fslbm_batch_step(h, n)
        close = lambda: F.fslbm_batch_destroy(h)
    else:
        b = F.Batch(doms, tuning_cache_path="")
        step, close = b.step, b.close
    step(27)
    doms[0].step(1)  # a member stepped alone: the batch rebuilds its tables
    step(18)
    close()
    out = [(d.read(KEYS), d.bubbles(), d.read(())["scalars"]) for d in doms]
    for d in doms:
        d.close()
    return out


def _same(a, b):
    for (ra, ba, sa), (rb, bb, sb) in zip(a, b):
        for k in KEYS:
            assert np.array_equal(ra[k], rb[k]), k
        for k in ba:
            assert np.array_equal(ba[k], bb[k]), k
        assert sa == sb


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_batch_equals_workspace_batch(prec):
    for big in (True, False):  # the second call on a smaller input
        ref = _run(_scenes(big), False, prec)
        got = _run(_scenes(big), True, prec)
        _same(ref, got)
        assert any(s["n_topology"] > 0 for _, _, s in ref) or not big


def test_noalloc_batch_rejects_what_does_not_fit():
    import paper_1604_01632_amd as F
    import torch
    d = F.Domain.from_scene(_scenes(False)[0], "fp32")
    with pytest.raises(F.FslbmError) as e:
        F.fslbm_batch_create_noalloc([d.handle] * 5000)
    assert e.value.code == F.FSLBM_EINVAL and "static batch tables" in str(e.value)
    other = torch.cuda.Stream()
    with pytest.raises(F.FslbmError) as e:
        F.fslbm_batch_create_noalloc([d.handle], stream=other)
    assert e.value.code == F.FSLBM_EINVAL and "stream" in str(e.value)
    d.close()

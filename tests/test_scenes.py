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

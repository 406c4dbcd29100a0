"""Comparison of the GPU library with the CPU oracle on the same scene."""
from __future__ import annotations

import sys

import numpy as np

import scenes

IFACE, LIQ = scenes.IFACE, scenes.LIQ

# FP64 form against the FP64 oracle.  Both compute every quantity with the
# same operation order and every per-cell sum exactly rounded, so the state
# must agree bit for bit (exact=True).  The total mass is a diagnostic that
# the GPU accumulates before the conversions: 1e-13 relative.  TOL64 is the
# documented fallback bound on PDFs, fill levels, masses and bubble values.
TOL64 = 1e-12
TOL_MASS = 1e-13


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_state(o, g, label: str, tol: float = TOL64, fields=True, exact=True) -> dict:
    """Assert that oracle o and GPU domain g hold the same state: bit for bit
    (exact) or within tol."""
    do = o.read()
    dg = g.read()
    N = o.N
    to, tg = do["cell_type"], dg["cell_type"]
    bad = np.nonzero(to != tg)[0]
    if len(bad):
        eps = o.params.get("eps_convert", 1e-2)
        ph = do["phi"][bad]
        margin = np.minimum(np.abs(ph - (1 + eps)), np.abs(ph + eps))
        raise AssertionError(f"{label}: {len(bad)} cell types differ, e.g. cells {bad[:5].tolist()} "
                             f"oracle {to[bad[:5]].tolist()} gpu {tg[bad[:5]].tolist()}; "
                             f"min threshold margin {margin.min():.3e}")
    assert np.array_equal(do["bubble_id"], dg["bubble_id"]), f"{label}: bubble IDs differ"
    out = {}
    if fields:
        fl = (to == IFACE) | (to == LIQ)
        fo = do["f"].reshape(19, N)[:, fl]
        fg = dg["f"].reshape(19, N)[:, fl]
        rel = np.max(np.abs(fg - fo) / np.abs(fo)) if fo.size else 0.0
        assert np.all(fo > 0), f"{label}: non-positive oracle PDF"
        assert rel <= tol, f"{label}: f differs by {rel:.3e}"
        if exact:
            assert np.array_equal(fo, fg), f"{label}: f not bitwise equal (max rel {rel:.3e})"
        it = to == IFACE
        for k in ("phi", "mass"):
            a, b = do[k][it], dg[k][it]
            err = np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-3)) if a.size else 0.0
            assert err <= tol, f"{label}: {k} differs by {err:.3e}"
            if exact:
                assert np.array_equal(a, b), f"{label}: {k} not bitwise equal ({err:.3e})"
            out[k] = err
        out["f"] = rel
    bo, bg = o.bubbles(), g.bubbles()
    assert bo["id"].tolist() == bg["id"].tolist(), f"{label}: bubbles {bo['id']} vs {bg['id']}"
    assert bo["n_cells"].tolist() == bg["n_cells"].tolist(), f"{label}: bubble cell counts"
    assert bo["flags"].tolist() == bg["flags"].tolist(), f"{label}: bubble flags"
    for k in ("volume", "v_star", "pressure"):
        err = np.max(np.abs(bo[k] - bg[k]) / np.maximum(np.abs(bo[k]), 1e-12)) if len(bo[k]) else 0.0
        assert err <= tol, f"{label}: bubble {k} differs by {err:.3e}"
        if exact:
            assert np.array_equal(bo[k], bg[k]), f"{label}: bubble {k} not bitwise equal ({err:.3e})"
        out["b_" + k] = err
    so, sg = o.scalars(), dg["scalars"]
    assert so["step"] == sg["step"] and so["next_id"] == sg["next_id"], f"{label}: scalars {so} {sg}"
    assert abs(so["total_mass"] - sg["total_mass"]) <= TOL_MASS * abs(so["total_mass"]), \
        f"{label}: total mass {so['total_mass']} vs {sg['total_mass']}"
    if exact:
        assert so["bucket"] == sg["bucket"], f"{label}: bucket {so['bucket']} vs {sg['bucket']}"
    else:
        assert abs(so["bucket"] - sg["bucket"]) <= tol * abs(so["total_mass"]), \
            f"{label}: bucket {so['bucket']} vs {sg['bucket']}"
    return out


def oracle_from_state(params: dict, state: dict, bubbles: dict, scalars: dict):
    """An oracle that continues from a saved state: the fields of a read
    (of the oracle or of a GPU domain), its bubble table and its step,
    next ID and bucket."""
    import oracle

    b = [(int(i), int(fl), float(vs), float(p))
         for i, fl, vs, p in zip(bubbles["id"], bubbles["flags"], bubbles["v_star"],
                                 bubbles["pressure"])]
    return oracle.Oracle(params, state["cell_type"], state["phi"], state["rho"], state["u"],
                         state["bubble_id"], b, f_init=state["f"], mass_init=state["mass"],
                         step0=scalars["step"], next_id0=scalars["next_id"],
                         bucket0=scalars["bucket"])


def run_pair(sc, steps: int, every: int, name: str, precision="fp64", **over):
    import oracle
    from paper_1604_01632_amd import Domain

    say(f"[parity] {name}: {sc.nx}x{sc.ny}x{sc.nz} steps={steps} every={every} {over}")
    o = oracle.Oracle.from_scene(sc, **over)
    g = Domain.from_scene(sc, precision, **over)
    exact = precision == "fp64"
    compare_state(o, g, f"{name} step 0", exact=exact)
    worst = {}
    done = 0
    while done < steps:
        k = min(every, steps - done)
        o.step(k)
        g.step(k)
        done += k
        r = compare_state(o, g, f"{name} step {done}", exact=exact)
        for key, v in r.items():
            worst[key] = max(worst.get(key, 0.0), v)
    s = o.scalars()
    say(f"[parity] {name}: ok ({'bitwise' if exact else 'within tolerance'}); worst {', '.join(f'{k}={v:.1e}' for k, v in worst.items())}; "
        f"topology changes {s['n_topology']}, bubbles {len(o.bubbles()['id'])}")
    return o, g

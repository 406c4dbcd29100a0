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


# One FP32 step from an FP32-representable state against the FP64 oracle.
# Every stored value is the result of a few dozen FP32 operations (unit
# roundoff 2^-24 = 6e-8) on terms of the size of the equilibrium
# populations, w_a rho: a PDF therefore carries an absolute error of a few
# ulp of w_a, whatever its own size (a reconstructed population can come
# out far below w_a), and agrees to 1e-5 relative to max(|f|, w_a).  Fill
# levels and masses (order one) agree to 1e-5 absolute.  Bubble volumes are
# exact sums of the fill levels (order 1e3 cells per bubble): 1e-6
# relative; V* and p follow them.  The total mass is the FP64 sum of FP32
# cell values: 1e-7 relative.
TOL_F = 1e-5
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
# Two discrete choices of an interface cell are taken on its normal n, in
# the precision of the form: which directions are reconstructed (c_a.n > 0)
# and the dominant axis of the height function.  Each component of n is a
# sum of 18 terms of size at most 4 |phi| (phi <= 1.1), so in FP32 it is off
# by at most about 18 * 2^-24 * 4.4 * 18 = 8.5e-5 in the worst case, and
# c_a.n or the gap between two |n_k| by twice that: within that band of a
# tie the FP32 form may choose the other way.  Only such a cell may hold
# PDFs beyond TOL_F (its other values are bounded as usual).
TIE_BAND = 2e-4
TOL_FIELD = 1e-5
TOL_BUBBLE = 1e-6
TOL_MASS32 = 1e-7


def near_tie(i, t_before, normal, c, shape):
    """Smallest distance of an FP64 decision of interface cell i from its
    tie: |c_a.n| over the directions whose source cell is interface or
    liquid, and the gap between the two largest |n_k|."""
    nz, ny, nx = shape
    n = normal[:, i]
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    d = np.inf
    for a in range(1, 19):
        sx, sy, sz = (x - c[a, 0]) % nx, (y - c[a, 1]) % ny, (z - c[a, 2]) % nz
        if t_before[sx + nx * (sy + ny * sz)] in (IFACE, LIQ):
            d = min(d, abs(float(c[a] @ n)))
    an = np.sort(np.abs(n))
    return min(d, float(an[2] - an[1]))


def compare_fp32_step(do, bo, so, dg, bg, sg, N, eps, audit):
    to, tg = do["cell_type"], dg["cell_type"]
    bad = np.nonzero(to != tg)[0]
    if bad.size:
        ph = do["phi"][bad]
        margin = np.minimum(np.abs(ph - (1 + eps)), np.abs(ph + eps))
        raise AssertionError(f"{bad.size} cell types differ, e.g. {bad[:5].tolist()}; "
                             f"min threshold margin {margin.min():.3e}")
    assert np.array_equal(do["bubble_id"], dg["bubble_id"]), "bubble IDs differ"
    fl = (to == IFACE) | (to == LIQ)
    cells = np.nonzero(fl)[0]
    fo, fg = do["f"].reshape(19, N), dg["f"].reshape(19, N)
    rel_f, worst, beyond = 0.0, None, np.zeros(cells.size, bool)
    for a in range(19):
        x, y = fo[a, fl], fg[a, fl]
        assert np.all(x > 0)
        e = np.abs(y - x) / np.maximum(x, W[a])
        beyond |= e > TOL_F
        e[beyond] = 0.0  # judged by the audit below
        k = int(np.argmax(e))
        if e[k] > rel_f:
            rel_f, worst = float(e[k]), (a, int(cells[k]), float(x[k]), float(y[k]))
    if worst is not None:
        a, i, x, y = worst
        say(f"[fp32 step] worst PDF within the bound: direction {a}, cell {i}, oracle {x:.9e}, "
            f"gpu {y:.9e}")
    odd = cells[beyond]
    ties = [audit(int(i)) for i in odd]
    say(f"[fp32 step] {odd.size} cell(s) with PDFs beyond {TOL_F:g}: types at t "
        f"{sorted(set(int(audit.t_before[i]) for i in odd))}, distance of an FP64 choice "
        f"from its tie at most {max(ties, default=0.0):.2e}")
    assert all(audit.t_before[i] == IFACE for i in odd)
    assert max(ties, default=0.0) <= TIE_BAND, "PDFs differ at a cell with no near-tie choice"
    assert odd.size <= max(1, cells.size // 100000)
    it = to == IFACE
    err = {k: float(np.max(np.abs(do[k][it] - dg[k][it]))) for k in ("phi", "mass")}
    assert bo["id"].tolist() == bg["id"].tolist(), "bubble IDs of the table differ"
    assert bo["n_cells"].tolist() == bg["n_cells"].tolist(), "bubble cell counts differ"
    assert bo["flags"].tolist() == bg["flags"].tolist()
    berr = {k: float(np.max(np.abs(bo[k] - bg[k]) / np.abs(bo[k]))) for k in
            ("volume", "v_star", "pressure")}
    merr = abs(so["total_mass"] - sg["total_mass"]) / abs(so["total_mass"])
    say(f"[fp32 step] fp32 step vs oracle: f {rel_f:.2e}, phi {err['phi']:.2e}, mass "
        f"{err['mass']:.2e}, bubbles {', '.join(f'{k} {v:.2e}' for k, v in berr.items())}, "
        f"total mass {merr:.2e}")
    assert rel_f <= TOL_F
    assert err["phi"] <= TOL_FIELD and err["mass"] <= TOL_FIELD
    for v in berr.values():
        assert v <= TOL_BUBBLE
    assert merr <= TOL_MASS32
    assert so["step"] == sg["step"] and so["next_id"] == sg["next_id"]


# Bubbles of two runs whose ID sequences differ (the forms see slightly
# different numbers of topology events) are paired by position.
def centroids(bid, ids, shape):
    """Centroid of every bubble's cells in the periodic box (circular mean
    per axis), in cell units."""
    nz, ny, nx = shape
    sel = bid >= 0
    cells = np.nonzero(sel)[0]
    lab = np.searchsorted(ids, bid[sel])
    out = np.zeros((len(ids), 3))
    for k, (n, coord) in enumerate(((nx, cells % nx), (ny, (cells // nx) % ny),
                                    (nz, cells // (nx * ny)))):
        a = 2 * np.pi * coord / n
        c = np.bincount(lab, np.cos(a), len(ids))
        s_ = np.bincount(lab, np.sin(a), len(ids))
        out[:, k] = (np.arctan2(s_, c) % (2 * np.pi)) * n / (2 * np.pi)
    return out


def match_by_centroid(ca, cb, shape):
    """For every bubble of a, the nearest bubble of b (periodic distance);
    None unless that is one to one."""
    L = np.array([shape[2], shape[1], shape[0]], float)
    d = np.abs(ca[:, None, :] - cb[None, :, :])
    d = np.minimum(d, L - d)
    m = np.argmin(np.sqrt((d ** 2).sum(-1)), axis=1)
    return m if len(set(m.tolist())) == len(m) else None

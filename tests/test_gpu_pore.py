"""The pore case (Sec. 3.2) on the GPU: the wetting rule (a static contact
angle in the height-function curvature at walls) and the open top (an
atmosphere bubble held at p0) against the oracle bit for bit in FP64, and
the detachment trend of the paper's table in FP32: a bubble pinches off
the pore, rises and joins the atmosphere, and a 70 degree contact angle
detaches a smaller bubble than 90 degrees."""
import numpy as np
import pytest

import scenes
from scenes import BUBBLE_ATMOSPHERE, BUBBLE_INLET, GAS, IFACE, LIQ

from tests.parity import run_pair, say

pytestmark = pytest.mark.gpu

P0 = scenes.P0


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


@pytest.mark.parametrize("theta,angle", [(60.0, 60.0), (120.0, 120.0), (90.0, 60.0), (90.0, 125.0)])
def test_wall_cap_matches_oracle(theta, angle):
    """A gas cap on a wall, at its own contact angle and off it (the contact
    line then moves): FP64 bit for bit with the oracle."""
    sc = scenes.wall_cap(theta, contact_angle=angle)
    run_pair(sc, 120, 40, f"cap {theta:g}/{angle:g}")


def _mini_pore(theta=70.0):
    return scenes.pore(r=3, n=(24, 24, 40), tau=0.6, top_gas=6, theta=theta, q_ml_min=1.0,
                       units=dict(g=2e-4, sigma=2e-3, q_per_ml_min=0.05))


def test_mini_pore_matches_oracle():
    """Inlet injection, wetting at the bottom and side walls and the
    atmosphere at the top together: FP64 bit for bit with the oracle."""
    sc = _mini_pore()
    o, g = run_pair(sc, 300, 100, "mini pore")
    b = g.bubbles()
    assert sorted(int(f) for f in b["flags"]) == [BUBBLE_INLET, BUBBLE_ATMOSPHERE]
    atm = [p for f, p in zip(b["flags"], b["pressure"]) if int(f) == BUBBLE_ATMOSPHERE]
    assert atm == [P0]


@pytest.mark.parametrize("first", [0, 1])
def test_joining_the_atmosphere_matches_oracle(first):
    spec = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, -0.08, 0)]
            + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
            + [(LIQ, 1.0, -1)] * 2)
    sc = scenes.layers(spec, ny=4, nz=4, p_init={0: P0 * 1.1, 1: P0 * 0.9})
    sc.bubbles = [(b, BUBBLE_ATMOSPHERE if b == first else f, v, p) for b, f, v, p in sc.bubbles]
    o, g = run_pair(sc, 3, 1, f"atmosphere merge {first}")
    b = g.bubbles()
    assert b["flags"].tolist() == [BUBBLE_ATMOSPHERE] and b["pressure"].tolist() == [P0]


def _detach(theta, r=6, q=10.0, max_steps=90000, after=0):
    """FP32 run of the similarity-mapped pore case to the first detachment;
    with `after` > 0 it goes on until the detached bubble has joined the
    atmosphere.  Returns (volume of the detached bubble in cells, steps,
    bubble table at the end)."""
    from paper_1604_01632_amd import Domain
    sc = scenes.pore(r=r, theta=theta, q_ml_min=q, tau=0.6, units=scenes.pore_units_similar(r))
    d = Domain.from_scene(sc, "fp32")
    done, vol = 0, None
    while done < max_steps:
        d.step(1000)
        done += 1000
        b = d.bubbles()
        free = [float(v) for f, v in zip(b["flags"], b["volume"]) if int(f) == 0]
        if free:
            vol = max(free)
            break
    assert vol is not None, f"no detachment in {max_steps} steps at {theta} degrees"
    t_detach = done
    while after and done < t_detach + after:
        d.step(1000)
        done += 1000
        b = d.bubbles()
        if not any(int(f) == 0 and float(v) > 0.5 * vol for f, v in zip(b["flags"], b["volume"])):
            break
    b = d.bubbles()
    say(f"[pore] theta {theta:g}: detached {vol:.0f} cells at step {t_detach}; end {done}: "
        f"{list(zip(b['id'].tolist(), b['flags'].tolist(), np.round(b['volume'], 1).tolist()))}")
    d.close()
    return vol, t_detach, done, b


def test_detachment_trend_and_rise_into_the_atmosphere():
    v70, t70, end, b = _detach(70.0, after=30000)
    # the detached bubble rose and joined the atmosphere: no free bubble of
    # its size is left, the atmosphere (p0) holds it and the pore grows a
    # new bubble that owns the inlet
    assert end < t70 + 30000
    atm = [i for i, f in enumerate(b["flags"]) if int(f) & BUBBLE_ATMOSPHERE]
    assert len(atm) == 1 and b["pressure"][atm[0]] == P0
    assert any(int(f) == BUBBLE_INLET for f in b["flags"])
    v90, t90, _, _ = _detach(90.0)
    # Table tab:detRad: a smaller detachment volume at 70 than at 90 degrees
    assert v70 < 0.85 * v90
    assert t70 < t90


def test_pore_checkpoint_restart():
    """Inlet, atmosphere and wetting through a checkpoint: 200 steps
    straight equal 100 steps, a readout through the boundary, a new domain
    from it and 100 more steps, bit for bit (FP64)."""
    from paper_1604_01632_amd import Domain
    sc = _mini_pore()
    a = Domain.from_scene(sc, "fp64")
    a.step(200)
    c = Domain.from_scene(sc, "fp64")
    c.step(100)
    ck = c.read()
    bub = c.bubbles()
    assert sorted(int(f) for f in bub["flags"]) == [BUBBLE_INLET, BUBBLE_ATMOSPHERE]
    binit = [(int(i), int(f), float(v), 0.0) for i, f, v in zip(bub["id"], bub["flags"], bub["v_star"])]
    d = Domain(sc.params(precision=0), ck["cell_type"], ck["phi"], ck["rho"], ck["u"], ck["bubble_id"],
               binit, f_init=ck["f"], restore=ck["scalars"], mass_init=ck["mass"])
    d.step(100)
    ra, rd = a.read(), d.read()
    for key in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(ra[key], rd[key]), key
    ba, bd = a.bubbles(), d.bubbles()
    for key in ba:
        assert np.array_equal(ba[key], bd[key]), key


def test_cap_relaxes_to_its_contact_angle():
    """A hemispherical gas cap (90 degrees) on a wall whose contact angle
    is 60, 90 or 120 degrees: the base contracts, stays, or spreads, to the
    base radius of the spherical cap of the same volume at that angle,
    a = Rs sin(theta) with V = pi Rs^3 (1 + cos)^2 (2 - cos) / 3, measured
    as the gas-region cells of the first fluid layer (an interface band of
    about half a cell beyond the contact line)."""
    from paper_1604_01632_amd import Domain
    radii = {}
    for ang in (60.0, 90.0, 120.0):
        sc = scenes.wall_cap(90.0, n=40, M=20, R=9.0, sigma=5e-3, contact_angle=ang)
        d = Domain.from_scene(sc, "fp32")
        d.step(3000)
        t = d.read(("cell_type",))["cell_type"].reshape(sc.nz, sc.ny, sc.nx)
        n = np.count_nonzero((t[1] == GAS) | (t[1] == IFACE))
        v = float(d.bubbles()["volume"][0])
        c = np.cos(np.radians(ang))
        rs = (3.0 * v / (np.pi * (1.0 + c) ** 2 * (2.0 - c))) ** (1.0 / 3.0)
        a = rs * np.sin(np.radians(ang))
        radii[ang] = (np.sqrt(n / np.pi), a)
        d.close()
    say(f"[pore] cap base radius (measured, cap of the same volume): {radii}")
    assert radii[60.0][0] < radii[90.0][0] < radii[120.0][0]
    for ang, (meas, exp) in radii.items():
        assert abs(meas - (exp + 0.5)) < 1.0, (ang, meas, exp)

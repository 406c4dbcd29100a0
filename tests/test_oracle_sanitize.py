"""The oracle built under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) runs small scenes with merges, splits, walls, gravity and
an inlet without a report, and computes exactly what the ordinary build
computes."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import scenes

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "oracle_san")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ORACLE_DIR, "sanitize_driver.c"), os.path.join(ORACLE_DIR, "fslbm_oracle.c"),
           "-I", ORACLE_DIR, "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    return exe, d


def _write_scene(path, sc, steps):
    p = sc.params()
    nb = len(sc.bubbles)
    with open(path, "wb") as f:
        f.write(struct.pack("<9i", sc.nx, sc.ny, sc.nz, *sc.periodic, 0, nb, steps))
        f.write(struct.pack("<9d", sc.tau, p["trt_lambda"], sc.sigma, *sc.g, p["p0"], sc.eps,
                            sc.inject_rate))
        f.write(np.ascontiguousarray(sc.cell_type, np.uint8).tobytes())
        for a in (sc.phi, sc.rho, sc.u):
            f.write(np.ascontiguousarray(a, np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.bubble_id, np.int32).tobytes())
        f.write(np.asarray([b[0] for b in sc.bubbles], np.int32).tobytes())
        f.write(np.asarray([b[1] for b in sc.bubbles], np.int32).tobytes())
        f.write(np.asarray([b[2] for b in sc.bubbles], np.float64).tobytes())
        f.write(np.asarray([b[3] for b in sc.bubbles], np.float64).tobytes())


def _read_out(path, N):
    b = open(path, "rb").read()
    o = 0

    def take(dtype, n):
        nonlocal o
        a = np.frombuffer(b, dtype=dtype, count=n, offset=o)
        o += a.nbytes
        return a

    out = dict(cell_type=take(np.uint8, N), phi=take(np.float64, N), mass=take(np.float64, N),
               f=take(np.float64, 19 * N), bubble_id=take(np.int32, N))
    out["step"] = int(take(np.int64, 1)[0])
    out["next_id"] = int(take(np.int32, 1)[0])
    out["bucket"] = float(take(np.float64, 1)[0])
    out["total_mass"] = float(take(np.float64, 1)[0])
    n = int(take(np.int32, 1)[0])
    rows = [(int(take(np.int32, 1)[0]), *take(np.float64, 3)) for _ in range(n)]
    out["bubbles"] = rows
    return out


P0 = scenes.P0
GAS, IFACE, LIQ = scenes.GAS, scenes.IFACE, scenes.LIQ
# an emptied film joins two bubbles; a filled neck splits one
MERGE = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, -0.08, 0)]
         + [(LIQ, 1.0, -1)] + [(IFACE, 0.5, 1)] + [(GAS, 0.0, 1)] * 3 + [(IFACE, 0.5, 1)]
         + [(LIQ, 1.0, -1)] * 2)
SPLIT = ([(LIQ, 1.0, -1)] * 3 + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 2 + [(IFACE, 0.5, 0)]
         + [(IFACE, 1.08, 0)] + [(IFACE, 0.5, 0)] + [(GAS, 0.0, 0)] * 3 + [(IFACE, 0.5, 0)]
         + [(LIQ, 1.0, -1)] * 3)

CASES = [
    # merges and splits within the horizon (three topology changes)
    ("blobs", lambda: scenes.merge_ids_if_touching(
        scenes.random_blobs(n=(21, 18, 17), nblob=4, seed=11, sigma=1e-2)), 80),
    ("walls-gravity", lambda: scenes.merge_ids_if_touching(
        scenes.random_blobs(n=(22, 19, 24), nblob=3, seed=7, walls=True, sigma=5e-3,
                            g=(0.0, 0.0, -2e-5))), 60),
    ("orifice", lambda: scenes.orifice(n=(14, 14, 20), r=3.0, Q=0.05, g=1e-4), 40),
    ("merge", lambda: scenes.layers(MERGE, ny=4, nz=4, p_init={0: P0 * 1.1, 1: P0 * 0.9}), 4),
    ("split", lambda: scenes.layers(SPLIT, ny=4, nz=4, p_init={0: P0 * 1.05}), 4),
]


@pytest.mark.parametrize("name,make,steps", CASES, ids=[c[0] for c in CASES])
def test_sanitized_oracle_matches(oracle_lib, driver, name, make, steps):
    exe, d = driver
    sc = make()
    scene_file, out_file = str(d / f"{name}.bin"), str(d / f"{name}.out")
    _write_scene(scene_file, sc, steps)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, scene_file, out_file], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    got = _read_out(out_file, sc.n)
    o = oracle_lib.Oracle.from_scene(sc)
    o.step(steps)
    ref = o.read()
    for k in ("cell_type", "bubble_id", "phi", "mass", "f"):
        assert np.array_equal(got[k], ref[k]), k
    s = o.scalars()
    if name in ("blobs", "walls-gravity", "merge", "split"):
        assert s["n_topology"] >= 1
    assert (got["step"], got["next_id"], got["bucket"], got["total_mass"]) == (
        s["step"], s["next_id"], s["bucket"], s["total_mass"])
    b = o.bubbles()
    assert [r[0] for r in got["bubbles"]] == list(b["id"])
    assert np.array_equal(np.array([r[1:] for r in got["bubbles"]]),
                          np.stack([b["volume"], b["v_star"], b["pressure"]], 1))

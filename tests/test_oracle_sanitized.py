"""The oracle's C++ under AddressSanitizer and UndefinedBehaviorSanitizer: a copy of
porta_oracle.cpp built with g++ -fsanitize=address,undefined (host code only) runs
every entry point on a small ragged problem in a child process with the sanitizer
runtimes preloaded; any report fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import dataclasses, sys
    import numpy as np
    sys.path.insert(0, {root!r})
    from paper_1307_4217_amd import inputs
    from oracle import oracle as orc
    assert orc.LIB == {lib!r}, orc.LIB
    cfg = inputs.Config("san", 6, 5, 9, 2, 3, 4, True)
    atm = dataclasses.replace(inputs.make_atmosphere(cfg, seed=3), lx=530.0, ly=410.0)
    q = inputs.make_quadrature(cfg)
    for interp in (0, 1):
        for control in (0, 1):
            out = orc.fs_sweep(orc.OracleProblem(atm, q, interp=interp, control=control))
            assert np.isfinite(out["jkq"]).all() and np.isfinite(out["itop"]).all()
    op = orc.OracleProblem(atm, q)
    n = atm.npoints
    rng = np.random.default_rng(0)
    _, im = orc.fs_sweep_cs(op, rng.normal(size=n), rng.normal(size=(6, n)),
                            rng.normal(size=(6, n)), h=1e-30, rays=[0, 3], freqs=[1, 2])
    assert np.isfinite(im).all()
    assert np.isfinite(orc.lc_sweep(op, [0, 5], [0, 3])).all()
    s, e, rc = orc.see_update(out["jkq"], atm.source, atm)
    op_s = orc.see_operator(out["jkq"], s, atm)
    assert np.isfinite(s).all() and np.isfinite(op_s).all()
    print("sanitized oracle ok")
""")


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    runtimes = [subprocess.run([gxx, f"-print-file-name={n}"], capture_output=True,
                               text=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(r) and os.path.exists(r) for r in runtimes):
        pytest.skip("sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fopenmp", "-fPIC", "-shared", "-Wall",
                           os.path.join(ROOT, "oracle", "porta_oracle.cpp"), "-o", lib])
    script = tmp_path / "run.py"
    script.write_text(SCRIPT.format(root=ROOT, lib=lib))
    env = dict(os.environ, LD_PRELOAD=":".join(runtimes), ASAN_OPTIONS="detect_leaks=0",
               PORTA_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env,
                       timeout=600, cwd=str(tmp_path))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr

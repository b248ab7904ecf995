"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and exercised on small grids in a child process: every
operator, the CG solve, the power method and explicit steps on a linear and a
saturating nonlinear workload must run without a sanitizer report (any
report aborts the child, which fails the test).  The results are also
checked against the regular build of the oracle, bitwise: the sanitized
build computes the same arithmetic (-O1 instead of -O3 changes no FP
operation order in these loops; compared to 1e-12 in case it does)."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys, json
    sys.path.insert(0, {root!r})
    import numpy as np
    import oracle, synth
    oracle.LIB_PATH = {lib!r}
    out = {{}}
    for name, wl in (("c1", synth.linear_c1(8)), ("nl", synth.nonlinear(8, ramp_steps=6, J0=6.0e6))):
        P = oracle.Problem(wl)
        rng = np.random.default_rng(3)
        x = rng.standard_normal(P.n_pad)
        y = P.kn(np.where(P.N, x, 0.0))
        lam = P.power(iters=20)
        dt = 0.5 * 2 / lam
        A, *_ = P.run(dt, 6, rtol=1e-12)
        s = P.cg(y, rtol=1e-12)[0]
        out[name] = [float(np.linalg.norm(y)), float(lam), float(np.linalg.norm(A)),
                     float(np.linalg.norm(s))]
    print("RESULT", json.dumps(out), flush=True)
""")


@pytest.mark.timeout(300)
def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libecoracle_san.so")
    src = os.path.join(ROOT, "oracle", "ec_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-o", lib,
                    src, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

    def child(libpath, extra_env):
        r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=libpath)],
                           capture_output=True, text=True, env=extra_env, timeout=280)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
            r.stderr[-4000:]
        line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
        import json
        return json.loads(line[len("RESULT "):])

    san = child(lib, env)
    import oracle
    plain_env = dict(os.environ, OMP_NUM_THREADS="2")
    plain = child(oracle.build(force=False), plain_env)
    for k in plain:
        for a, b in zip(san[k], plain[k]):
            assert abs(a - b) <= 1e-12 * max(abs(b), 1e-300), (k, san[k], plain[k])

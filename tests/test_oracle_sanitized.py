"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run on small cases of every entry point: brute
force under both cutoffs and all cell sets, the per-molecule evaluation with
a sample, the linked-cell evaluation with a base-cell range, binning and the
single-triplet helpers.  Any out-of-bounds access, leak or undefined
operation aborts the child process."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    src = os.path.join(ROOT, "oracle", "atm3_oracle.c")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                           src, "-lm"])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        import oracle
        oracle._LIB = {str(lib)!r}
        oracle._lib = None
        from paper_2510_21230_amd import workloads
        pos, box = workloads.uniform(160, [8.0, 8.0, 8.0], seed=3)
        for tr in ("pair", "product"):
            for var in ("3c08", "3c18", "3c01"):
                if tr == "product" or var == "3c08":
                    L = 13.0 if var == "3c18" else 8.0
                    p, b = workloads.uniform(160, [L, L, L], seed=4)
                    a = oracle.brute(p, b, truncation=tr, variant=var)
                    m = oracle.molecules(p, b, truncation=tr, variant=var, sample=np.array([0, 5, 159]))
        c = oracle.cells(pos, box)
        h = oracle.cells(pos, box, base_cells=(0, 10))
        w = oracle.virial_diag(pos, box)
        cxyz, clin, nc = oracle.bin_cells(pos, box, 2.5)
        oracle.triplet(np.array([1.0, 0, 0]), np.array([0, 1.1, 0]), np.array([-1.0, 1.1, 0]), 0.073)
        print("ok", a.n_triplets, c.n_triplets)
    """)
    # the sanitizer runtimes go first in the preload list; anything already
    # preloaded stays loaded after them
    pre = [p for p in (asan, ubsan) if os.path.isabs(p)]
    if os.environ.get("LD_PRELOAD"):
        pre.append(os.environ["LD_PRELOAD"])
    env = dict(os.environ, LD_PRELOAD=" ".join(pre), ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]

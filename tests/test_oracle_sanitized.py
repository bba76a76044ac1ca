"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
CPU only): every entry point (log Z, marginals with the reverse pass, the
sampler) runs on small proteins, including one- and two-residue edge cases
and a loop-rich model, with no sanitizer report, and gives the log Z of the
regular build."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2604_19718_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ORC = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", exe,
           os.path.join(ORC, "oracle.c"), os.path.join(ORC, "seqmcc.c"),
           os.path.join(ORC, "sanitize_driver.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("gcc sanitizer build unavailable: " + r.stderr[-400:])
    return exe


@pytest.mark.parametrize("case", [("M", 5), ("KW", 5), ("GASRL", 20), ("CYHWMKLV", 20), ("interior", 10)])
def test_entry_points_clean_under_sanitizers(driver, tmp_path, case):
    prot, ns = case
    if prot == "interior":
        prot = "GCAGRLVK"
        en = I.interior_rich_energy(11)
    else:
        en = I.energy_tables(1001)
    m = len(prot)
    t1 = I.theta1(5, prot, 0.5)
    t2 = I.theta2(5, prot, 0.3)
    path = str(tmp_path / "prob.bin")
    np.concatenate([en.packed(), t1.ravel(), t2.ravel()]).astype(np.float64).tofile(path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="1")
    r = subprocess.run([driver, path, prot, str(ns)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-2000:]
    lz1, lz2, rc = r.stdout.split()
    ref = oracle.logz(I.Problem(prot, t1, t2), en)
    assert int(rc) == 0
    assert abs(float(lz1) - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(float(lz2) - ref) <= 1e-12 * max(1.0, abs(ref))

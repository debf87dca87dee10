"""The C ABI from a plain C program.

CPU: tests/c/count_dd.c compiles as C99 against include/tpcf.h alone and
links against libtpcf.so (the header is valid C and declares what the
library exports).  GPU: the program counts DD for a small catalog with every
precision, and the counts equal the oracle's.
"""

import os
import subprocess

import numpy as np
import pytest

import oracle
import paper_1204_6630_amd as tp
import synthcat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "count_dd.c")
LIBDIR = os.path.dirname(tp.lib_path())


def _build(tmp_path):
    exe = str(tmp_path / "count_dd")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I" + os.path.join(ROOT, "include"),
                           SRC, "-o", exe, "-L" + LIBDIR, "-ltpcf", "-Wl,-rpath," + LIBDIR])
    return exe


def test_c_client_compiles_and_links(tmp_path):
    if not os.path.exists(tp.lib_path()):
        pytest.skip("libtpcf.so is not built")
    # the library is linked by its file name
    link = os.path.join(LIBDIR, "libtpcf.so")
    assert os.path.exists(link)
    assert os.path.exists(_build(tmp_path))


@pytest.mark.gpu
def test_c_client_counts_equal_the_oracle(tmp_path):
    exe = _build(tmp_path)
    wl = synthcat.patch30_1e4(scale=0.1)
    d = wl.data[0]
    e = wl.edges_deg
    lines = ([str(d.n)] + [f"{float(a)!r} {float(b)!r}" for a, b in zip(d.ra, d.dec)] + [str(e.size - 1)]
             + [repr(float(x)) for x in e])
    # the library shares torch's HIP runtime when loaded from Python; a C
    # program loads the system one
    r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = [np.array([int(v) for v in line.split()], dtype=np.uint64) for line in r.stdout.strip().splitlines()]
    ref = oracle.count(oracle.DD, oracle.radec_to_xyz(d.ra, d.dec), e)
    assert len(got) == 2
    for g in got:
        assert np.array_equal(g, ref)

"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The library's forest topology (csrc/topology.cpp: leaf table, refine,
  2:1 corner balance, coarsen and the remap lists of Sec. 2.2) is built with
  g++ -fsanitize=address,undefined together with a small driver
  (tests/sanitize/topology_driver.cpp) and run on random regrid sequences
  (2D and 3D, bricks of 1 to 3 trees per axis, periodic and bounded axes);
  its leaf tables and remap lists must equal the oracle forest's, and any
  sanitizer report fails the run.
* The C oracle is built with the same sanitizers and the oracle's ghost,
  pattern, regrid and boundary pins run against it in a child process."""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

from oracle.mesh import Forest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_07612_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV_SAN = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


@pytest.fixture(scope="module")
def topo_driver(tmp_path_factory):
    _need("g++")
    exe = str(tmp_path_factory.mktemp("san") / "topology_driver")
    cmd = ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                                         os.path.join(CSRC, "topology.cpp"),
                                         os.path.join(ROOT, "tests", "sanitize", "topology_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot build the topology driver: " + r.stderr[-800:])
    return exe


def _random_flags(rng, nb):
    return rng.choice([-1, 0, 0, 1], size=nb, p=[0.45, 0.25, 0.1, 0.2]).astype(np.int8)


CASES = [(2, (1, 1, 1), (1, 1, 1)), (2, (3, 2, 1), (1, 0, 1)), (3, (2, 2, 2), (1, 1, 1)),
         (3, (1, 2, 3), (0, 1, 1)), (3, (2, 1, 1), (0, 0, 0))]


@pytest.mark.parametrize("ndim,nt,per", CASES, ids=[f"{c[0]}d-{c[1]}-{c[2]}" for c in CASES])
def test_topology_under_sanitizers_equals_oracle_forest(topo_driver, ndim, nt, per):
    rng = np.random.default_rng(sum(nt) * 7 + ndim + 31 * sum(per))
    lmin, lmax, init = 0, 3, 1
    forest = Forest(ndim, nt, periodic=[bool(p) for p in per], level=init)
    script = [f"{ndim} {nt[0]} {nt[1]} {nt[2]} {per[0]} {per[1]} {per[2]} {init} {lmin} {lmax} 6"]
    expected = []
    for _ in range(6):
        flags = _random_flags(rng, forest.nb)
        script.append(f"{forest.nb} " + " ".join(str(int(f)) for f in flags))
        res = forest.regrid(flags, lmin, lmax)
        if res is None:
            expected.append(None)
        else:
            op, src, arg = res
            expected.append([(l, *G, int(o), int(s), int(a)) for (l, G), o, s, a in zip(forest.leaves, op, src, arg)])
    r = subprocess.run([topo_driver], input="\n".join(script) + "\n", capture_output=True, text=True,
                       env=dict(os.environ, **ENV_SAN), timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.splitlines()
    i = 1 + int(lines[0].split()[1])  # skip the initial table
    for want in expected:
        _, changed, nb = lines[i].split()
        i += 1
        if want is None:
            assert changed == "0"
            continue
        assert changed == "1" and int(nb) == len(want)
        got = [tuple(int(x) for x in lines[i + k].split()) for k in range(len(want))]
        i += len(want)
        assert got == [tuple(int(x) for x in w) for w in want]


@pytest.fixture(scope="module")
def sanitized_oracle(tmp_path_factory):
    _need("gcc")
    so = str(tmp_path_factory.mktemp("san") / "libfoap4_oracle_san.so")
    cmd = ["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared"] + SAN + \
        [os.path.join(ROOT, "oracle", "foap4_oracle.c"), "-o", so, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot build the sanitized oracle: " + r.stderr[-800:])
    return so


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_pins_under_sanitizers(sanitized_oracle):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not found")
    sel = ("pattern or regrid or ghost or prolong or restrict or appendix or linear or uniform_state "
           "or flux_fix or boundar or dirichlet or wall or bc_data")
    env = dict(os.environ, FOAP4_ORACLE_LIB=sanitized_oracle, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               **ENV_SAN)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-k", sel,
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_boundaries.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    tail = (r.stdout[-2000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert " passed" in r.stdout, tail

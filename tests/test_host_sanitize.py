"""Host planning code under AddressSanitizer and UndefinedBehaviorSanitizer
(code safety: bounds checking and graceful handling of bad input, Girder 1,
"Code safety").

The planner, tile choice, planner dry run, tile-table reader, object
registry and indexing-vector bounds check are compiled with g++
-fsanitize=address,undefined (host code only: no HIP source is part of this
build) into a small driver (tests/sanitize/driver.cpp), which runs a battery
of valid and invalid descriptors.  Any sanitizer report aborts the driver;
its results must equal those of the regular library on the same cases.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_07311_amd", "csrc")
HOST_SOURCES = ["planner.cpp", "plan_host.cpp", "table.cpp", "registry.cpp"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("sanitize") / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, os.path.join(ROOT, "tests", "sanitize", "driver.cpp")] + \
        [os.path.join(CSRC, s) for s in HOST_SOURCES] + ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def run(driver, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver] + list(args), capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, "driver failed (%d):\n%s\n%s" % (r.returncode, r.stdout, r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.fixture(scope="module")
def fm():
    import paper_2604_07311_amd as fm
    if not os.path.exists(fm.LIB_PATH):
        from paper_2604_07311_amd import build
        build.build()
    fm.load_library()
    return fm


def _cases():
    """(dtype, compute, [(extents, strides, labels)] * 3) for valid and
    invalid descriptors."""
    out = []

    def add(p, dtypes=(1, 2), computes=(0,)):
        for dt in dtypes:
            for cp in computes:
                if cp and dt != 2:
                    continue
                out.append((dt, cp, [(t.extents, t.strides, [ord(c) for c in lab])
                                     for t, lab in ((p.a, p.la), (p.b, p.lb), (p.c, p.lc))]))
    add(synth.plain16(with_data=False), computes=(0, 1, 2))
    add(synth.ladder(128, 32, with_data=False), computes=(0, 1, 2))
    add(synth.ladder(192, 48, with_data=False), computes=(0, 1))
    add(synth.ring(48, 192, with_data=False), computes=(0, 1, 2))
    add(synth.autograd_case(24, 96, with_data=False))
    rng = np.random.default_rng(77)
    for _ in range(40):
        add(synth.random_problem(rng, 1, 9), computes=(0, 1))

    def raw(dt, cp, la, ea, sa, lb, eb, sb, lc, ec, sc):
        out.append((dt, cp, [(ea, sa, [ord(c) for c in la]), (eb, sb, [ord(c) for c in lb]),
                             (ec, sc, [ord(c) for c in lc])]))
    raw(1, 0, "ik", [2, 3], [1, 2], "kj", [4, 5], [1, 4], "ij", [2, 5], [1, 2])      # shape mismatch
    raw(1, 0, "ik", [2, 3], [1, 2], "kj", [3, 5], [1, 3], "iz", [2, 5], [1, 2])      # label
    raw(1, 0, "ik", [2, 3], [1, 2], "kj", [3, 2], [1, 3], "ii", [2, 2], [1, 2])      # repeated in C
    raw(1, 0, "ik", [2, 3], [1, 2], "kj", [3, 2], [1, 3], "ij", [2, 2], [1, 1])      # C not injective
    raw(7, 0, "ik", [2, 3], [1, 2], "kj", [3, 2], [1, 3], "ij", [2, 2], [1, 2])      # bad dtype
    raw(1, 1, "ik", [2, 3], [1, 2], "kj", [3, 2], [1, 3], "ij", [2, 2], [1, 2])      # bf16x3 on FP64
    raw(2, 9, "ik", [2, 3], [1, 2], "kj", [3, 2], [1, 3], "ij", [2, 2], [1, 2])      # bad compute
    raw(1, 0, "ik", [2, -3], [1, 2], "kj", [3, 2], [1, 3], "ij", [2, 2], [1, 2])     # negative extent
    raw(1, 0, "abcdefghi", [1] * 9, [1] * 9, "j", [2], [1], "j", [2], [1])           # rank 9
    raw(2, 0, "k", [5], [1], "k", [5], [2], "", [], [])                               # dot product
    raw(2, 0, "ik", [3, 0], [1, 3], "kj", [0, 2], [1, 1], "ij", [3, 2], [1, 3])      # K = 0
    raw(2, 0, "ik", [0, 4], [1, 1], "kj", [4, 2], [1, 4], "ij", [0, 2], [1, 1])      # M = 0
    raw(1, 0, "ik", [3, 4], [-1, 3], "kj", [4, 5], [1, 0], "ij", [3, 5], [5, 1])     # negative / zero strides
    raw(1, 0, "iik", [3, 3, 4], [1, 3, 9], "kj", [4, 2], [1, 4], "ij", [3, 2], [1, 3])  # diagonal
    raw(1, 0, "itk", [3, 5, 4], [1, 3, 15], "kj", [4, 2], [1, 4], "ij", [3, 2], [1, 3])  # summed in A
    raw(1, 0, "lik", [2, 3, 4], [1, 2, 6], "lkj", [2, 4, 2], [1, 2, 8], "lij", [2, 3, 2], [1, 2, 6])  # batch
    raw(1, 0, "abcdefgh", [2] * 8, [1, 2, 4, 8, 16, 32, 64, 128], "abcdefgh", [2] * 8,
        [128, 64, 32, 16, 8, 4, 2, 1], "", [], [])                                    # rank 8, full contraction
    raw(1, 0, "ik", [1 << 40, 2], [1, 1 << 40], "kj", [2, 2], [1, 2], "ij", [1 << 40, 2], [1, 1 << 40])  # huge M
    return out


def _expected(fm, case):
    dt, cp, ts = case
    d = [fm.make_desc(e, s, l) for e, s, l in ts]
    try:
        info, offs = fm.famlies_analyze(dt, cp, *d, want_offsets=True)
    except fm.FamliesError as e:
        return "%d" % e.code
    vec = np.concatenate([offs[k] for k in ("xrow", "xk", "yk", "ycol", "crow", "ccol",
                                             "xbatch", "ybatch", "cbatch")])
    s = 0
    for i, v in enumerate(vec.tolist()):
        s = (s + (v % (1 << 64)) * (i % 97 + 1)) % (1 << 64)
    f = ["m", "n", "k", "batch", "swapped", "x_kfast", "y_kfast", "n_i", "n_j", "n_p", "n_batch",
         "n_trace", "n_diag", "tile_m", "tile_n", "tile_k", "split_k", "index_bits", "kernel",
         "split_tiles", "index_elements"]
    return " ".join(["0"] + [str(int(info[k])) for k in f] + [str(s)])


def test_analyze_under_sanitizers_matches_library(driver, fm, tmp_path):
    cases = _cases()
    path = tmp_path / "cases.txt"
    with open(path, "w") as f:
        for dt, cp, ts in cases:
            parts = [dt, cp]
            for e, s, l in ts:
                parts += [len(e)] + list(e) + list(s) + list(l)
            f.write(" ".join(str(int(x)) for x in parts) + "\n")
    got = run(driver, "analyze", str(path)).splitlines()
    assert len(got) == len(cases)
    n_err = 0
    for case, line in zip(cases, got):
        want = _expected(fm, case)
        assert line == want, (case, line, want)
        n_err += line.split()[0] != "0"
    assert 8 <= n_err < len(cases)


def test_tile_table_reader_under_sanitizers(driver, tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("# comment\nplain 1 0 10 10 14 128 128 16 1\nbatch 2 0 6 6 10 64 64 32 1 0\n"
                    "plain 2 0 12 8 12 128 128 32 3 64 72\n\n")
    assert run(driver, "table", str(good)).strip() == "ok 3"
    for bad in ["plain 1 0 10 10 14 128 128 16\n", "dense 1 0 1 1 1 128 128 16 1\n",
                "plain 1 0 1 1 1 -128 128 16 1\n", "plain 1 0 1 1 1 128 128 16 1 48\n",
                "plain 1 0 1 1 1 128 128 16 2 0 -1\n", "plain x y z\n",
                "plain 1 0 1 1 1 99999999999999999999 128 16 1\n"]:
        p = tmp_path / "bad.txt"
        p.write_text(bad)
        assert run(driver, "table", str(p)).strip() == "err", bad
    assert run(driver, "table", str(tmp_path / "missing.txt")).strip() == "err"


def test_registry_under_sanitizers(driver):
    assert run(driver, "registry").strip() == "registry ok"


def test_bounds_check_under_sanitizers(driver):
    # inside, one past the end, before the start, negative strides, nothing
    # addressed, vector shorter than claimed
    assert run(driver, "bounds").split() == ["1", "0", "0", "1", "1", "0"]

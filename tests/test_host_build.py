"""Host build of the library's per-lane algebra under AddressSanitizer and
UndefinedBehaviorSanitizer, checked against the oracle.

tests/host_build/element_check.cpp compiles the device headers (linalg.hpp,
operators.hpp, sqrt.hpp, elements.hpp) for the CPU through a small stand-in
for the HIP runtime header, with g++ -fsanitize=address,undefined and no
recovery, so any out-of-bounds access or undefined operation in the unrolled
register algebra aborts the run.  For seeded random operands it evaluates, in
the matrix form and in the lower-triangular factor form, the filtering
element (eq. 13-14), the filtering operator and its carry application
(eq. 15), the smoothing element (eq. 17) and the smoothing operator (eq. 19);
each result must equal the oracle's evaluation of the same equation.  This
covers the element algebra only: cross-lane shuffles, LDS and the kernels'
launch geometry are not modelled on the host.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2102_00514_amd", "csrc")

TOL = {"f64": 1e-12, "f32": 2e-5}


@pytest.fixture(scope="module")
def cases(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("host_build") / "element_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wno-unknown-pragmas", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(HERE, "host_build", "shim"), "-I", CSRC,
           "-o", exe, os.path.join(HERE, "host_build", "element_check.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe, "20260", "12"], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
    return [json.loads(line) for line in res.stdout.splitlines()]


def _a(r, k, shape):
    return np.array(r[k], dtype=np.float64).reshape(shape)


def _filter_pack(r, s, n):
    return np.concatenate([_a(r, "A" + s, (n, n)).ravel(), _a(r, "b" + s, (n,)), _a(r, "C" + s, (n, n)).ravel(),
                           _a(r, "eta" + s, (n,)), _a(r, "J" + s, (n, n)).ravel()])


def _reference(r):
    n, p = r["n"], r["p"]
    kind = r["kind"]
    if kind == "filter_element":
        e = oracle.filter_element(_a(r, "F", (n, n)), _a(r, "c", (n,)), _a(r, "Qp", (n, n)), _a(r, "H", (p, n)),
                                  _a(r, "d", (p,)), _a(r, "Rp", (p, p)), _a(r, "y", (p,)))
        return dict(zip(("A", "b", "C", "eta", "J"), oracle.unpack_filter(e, n)))
    if kind == "filter_combine":
        e = oracle.filter_combine(_filter_pack(r, "i", n), _filter_pack(r, "j", n), n)
        return dict(zip(("A", "b", "C", "eta", "J"), oracle.unpack_filter(e, n)))
    if kind == "filter_apply":
        # a carry is the element (0, b, C, 0, 0)
        ai = np.concatenate([np.zeros(n * n), _a(r, "bi", (n,)), _a(r, "Ci", (n, n)).ravel(), np.zeros(n),
                             np.zeros(n * n)])
        e = oracle.filter_combine(ai, _filter_pack(r, "j", n), n)
        A, b, C, _, _ = oracle.unpack_filter(e, n)
        return {"b": b, "C": C}
    if kind == "smoother_element":
        e = oracle.smoother_element(_a(r, "x", (n,)), _a(r, "P", (n, n)), _a(r, "F", (n, n)), _a(r, "c", (n,)),
                                    _a(r, "Qp", (n, n)))
    else:
        ai = np.concatenate([_a(r, "Ei", (n, n)).ravel(), _a(r, "gi", (n,)), _a(r, "Li", (n, n)).ravel()])
        aj = np.concatenate([_a(r, "Ej", (n, n)).ravel(), _a(r, "gj", (n,)), _a(r, "Lj", (n, n)).ravel()])
        e = oracle.smoother_combine(ai, aj, n)
    nn = n * n
    return {"E": e[:nn].reshape(n, n), "g": e[nn:nn + n], "L": e[nn + n:].reshape(n, n)}


def test_runs_clean_and_covers_every_operation(cases):
    kinds = {(r["kind"], r["n"], r["prec"]) for r in cases}
    for k in ("filter_element", "filter_combine", "filter_apply"):
        assert {(k, 5, "f64"), (k, 3, "f64"), (k, 1, "f64"), (k, 5, "f32")} <= kinds
    for k in ("smoother_element", "smoother_combine"):
        assert {(k, 5, "f64"), (k, 3, "f64"), (k, 5, "f32")} <= kinds
    assert all(r.get("ok", True) for r in cases)


@pytest.mark.parametrize("form", ["cov", "sq"])
def test_forms_equal_the_oracle(cases, form):
    worst = {}
    for r in cases:
        for name, ref in _reference(r).items():
            got = _a(r, f"{form}_{name}", ref.shape)
            err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
            key = (r["kind"], r["n"], r["prec"], name)
            worst[key] = max(worst.get(key, 0.0), err)
            assert err <= TOL[r["prec"]], (form, key, err)
    print(form, max(v for k, v in worst.items() if k[2] == "f64"), max(v for k, v in worst.items() if k[2] == "f32"))


def test_factors_are_lower_triangular_with_nonnegative_diagonal(cases):
    for r in cases:
        n = r["n"]
        for k in ("sq_U", "sq_Z", "sq_D"):
            if k in r:
                L = _a(r, k, (n, n))
                assert np.all(np.triu(L, 1) == 0.0) and np.all(np.diag(L) >= 0.0), (r["kind"], k)

"""The squared-exponential constants compiled into the library (csrc/spingp_sqexp_tables.hpp):
they must reproduce the matrix exponential and the stationary covariance of the unit-lengthscale
companion matrix, built here with numpy and scipy from the spectral approximation (the inverse
spectral density truncated after order + 1 terms of its exponential series, its stable roots;
the paper allows a state-space form that approximates the kernel, Sec. 2.2, and uses the EQ
kernel in its CO2 model, Sec. 4.3), and match what the committed generator writes."""
import math
import os
import re
import sys

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1610_08035_amd", "csrc", "spingp_sqexp_tables.hpp")


ORDERS = (2, 4, 6, 8, 10)


def _read(n):
    """Roots, projectors and P1 of order n from the header."""
    txt = open(HEADER).read()

    def arr(name, kind=float):
        m = re.search(name + r"\[(\d+)\] = \{([^}]*)\}", txt)
        vals = np.array([kind(x) for x in m.group(2).split(",")])
        assert vals.size == int(m.group(1))
        return vals

    assert int(re.search(r"kSqExpMaxOrder = (\d+);", txt).group(1)) == max(ORDERS)
    q = n // 2 - 1
    r0, z0, p0 = (int(arr(a, int)[q]) for a in ("kSqExpRootOff", "kSqExpZOff", "kSqExpP1Off"))
    roots = (arr("kSqExpRootRe") + 1j * arr("kSqExpRootIm"))[r0:r0 + n // 2]
    Z = (arr("kSqExpZRe") + 1j * arr("kSqExpZIm"))[z0:z0 + n * n * (n // 2)].reshape(n, n, n // 2)
    return n, roots, Z, arr("kSqExpP1")[p0:p0 + n * n].reshape(n, n)


def _companion(n):
    # stable roots of sum_m (-r^2 / 2)^m / m!, m = 0..n
    u = np.roots([1.0 / math.factorial(k) for k in range(n, -1, -1)])
    r = np.sqrt(-2.0 * u.astype(complex))
    r = np.where(r.real < 0, r, -r)
    c = np.real(np.poly(r))
    C = np.diag(np.ones(n - 1), 1)
    C[-1, :] = -c[1:][::-1]
    return C, r


@pytest.mark.parametrize("order", ORDERS)
def test_roots_are_the_stable_upper_half(order):
    n, roots, _, _ = _read(order)
    _, r = _companion(n)
    want = np.sort_complex(r[r.imag > 0])
    assert np.allclose(np.sort_complex(roots), want, rtol=1e-12, atol=0)
    assert np.all(roots.real < 0) and np.all(roots.imag > 0)


@pytest.mark.parametrize("order", ORDERS)
def test_projectors_give_the_matrix_exponential(order):
    n, roots, Z, _ = _read(order)
    C, _ = _companion(n)
    for x in (0.0, 1e-4, 0.05, 0.7, 2.5, 9.0):
        E = 2.0 * np.real(np.einsum("rck,k->rc", Z, np.exp(roots * x)))
        assert np.abs(E - scipy.linalg.expm(C * x)).max() <= 1e-15 * max(1.0, np.abs(Z).sum(axis=2).max()) * n, x
    # the projectors sum to the identity and are idempotent
    # the projectors sum to the identity and are idempotent, up to the rounding of the entries
    # (their magnitudes grow with the order: sum |Z_k| is 2 at order 2 and 2e7 at order 10)
    full = 2.0 * np.real(Z.sum(axis=2))
    scale = np.abs(Z).sum(axis=2).max()
    assert np.abs(full - np.eye(n)).max() <= 4e-16 * scale
    for k in range(n // 2):
        zk = np.abs(Z[:, :, k]).max()
        assert np.abs(Z[:, :, k] @ Z[:, :, k] - Z[:, :, k]).max() <= 4e-16 * n * zk * zk


@pytest.mark.parametrize("order", ORDERS)
def test_stationary_covariance(order):
    n, _, _, P1 = _read(order)
    C, _ = _companion(n)
    kappa = math.sqrt(2.0 * math.pi) * math.factorial(n) * 2.0 ** n
    W = np.zeros((n, n))
    W[-1, -1] = kappa
    res = C @ P1 + P1 @ C.T + W
    assert np.abs(res).max() <= 1e-11 * kappa * max(1.0, np.abs(P1).max() / 1e4)
    assert np.allclose(P1, P1.T, rtol=1e-15, atol=0)
    assert np.all(np.linalg.eigvalsh(P1) > 0)
    # the implied kernel at lag 0 approaches 1 as the order grows (the truncation error: about
    # 0.3 % at order 6)
    err = {2: 0.15, 4: 0.02, 6: 3.1e-3, 8: 7e-4, 10: 1.5e-4}[n]
    assert abs(P1[0, 0] - 1.0) < err


@pytest.mark.parametrize("order", ORDERS)
def test_header_matches_the_generator(order):
    sys.path.insert(0, os.path.join(ROOT, "paper_1610_08035_amd"))
    try:
        from gen_sqexp_tables import tables
    finally:
        sys.path.pop(0)
    n, roots, Z, P1 = _read(order)
    r2, Z2, P2 = tables(n)
    assert np.array_equal(roots, r2) and np.array_equal(Z, Z2) and np.array_equal(P1, P2)

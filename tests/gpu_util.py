"""Shared helpers of the GPU parity tests (comparison bars and device transfer)."""
from __future__ import annotations

import numpy as np

# Bars (FP64).  mean: |dm| <= 1e-9 (|m| + sqrt(v)); variance: |dv| <= 1e-9 v; logML: 1e-8 relative;
# gradient: 1e-7 relative per component with a floor of 1e-3 * max|g| (components that are
# nearly zero by cancellation are compared on the scale of the largest one).
TOL_MEAN = 1e-9
TOL_VAR = 1e-9
TOL_LOGML = 1e-8
TOL_GRAD = 1e-7


def to_dev(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


def check_logml(got, ref, tol=TOL_LOGML):
    err = abs(got - ref) / abs(ref)
    assert err <= tol, f"logML {got!r} vs {ref!r}: rel {err:.3e} > {tol:g}"


def check_mean_var(fm, fv, ref_m, ref_v):
    scale = np.abs(ref_m) + np.sqrt(np.maximum(ref_v, 0.0))
    em = np.abs(fm - ref_m) / scale
    ev = np.abs(fv - ref_v) / ref_v
    i, j = int(np.argmax(em)), int(np.argmax(ev))
    assert em[i] <= TOL_MEAN, f"mean at {i}: {fm[i]!r} vs {ref_m[i]!r} ({em[i]:.3e})"
    assert ev[j] <= TOL_VAR, f"variance at {j}: {fv[j]!r} vs {ref_v[j]!r} ({ev[j]:.3e})"


def check_grad(g, ref, tol=TOL_GRAD):
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    err = np.abs(g - ref) / scale
    assert err.max() <= tol, f"gradient {g} vs {ref}: rel {err.max():.3e} > {tol:g}"


def compare_series(terms, t, y, hyp, got, blocks=True, widen=1.0):
    """Element-wise comparison of one series' outputs with the C oracle.  `got` holds numpy
    arrays sliced to the series (f_mean, f_var, z_mean [b, n], S_diag [b(b+1)/2, n], S_sub
    [b*b, n]) and scalars (logml, logml2, datafit, logdet, grad [3], status); `widen`
    multiplies the mean/variance/block bars (1 = the 1e-9 bars)."""
    from oracle import native
    ref = native.btd_factored(terms, hyp, t, y, want_blocks=blocks)
    gref = native.tangent_grad(terms, hyp, t, y)
    assert got["status"] == 0
    check_logml(got["logml"], ref["logml"])
    check_logml(got["logml2"], ref["logml"])
    check_logml(got["datafit"], ref["datafit"], tol=1e-8)
    assert abs(got["logdet"] - ref["logdet"]) <= 1e-8 * max(1.0, abs(ref["logdet"]))
    tol = 1e-9 * widen
    sc_m = np.abs(ref["f_mean"]) + np.sqrt(ref["f_var"])
    assert np.max(np.abs(got["f_mean"] - ref["f_mean"]) / sc_m) <= tol
    assert np.max(np.abs(got["f_var"] - ref["f_var"]) / ref["f_var"]) <= tol
    if widen == 1.0:
        check_mean_var(got["f_mean"], got["f_var"], ref["f_mean"], ref["f_var"])
    check_grad(got["grad"], gref["grad"])
    if blocks:
        b = ref["z_mean"].shape[1]
        zs = np.sqrt(np.maximum(np.einsum("nii->ni", ref["S_diag"]), 0.0))
        ez = np.abs(got["z_mean"].T - ref["z_mean"]) / (np.abs(ref["z_mean"]) + zs)
        assert ez.max() <= tol, f"z_mean {ez.max():.3e} at {np.unravel_index(ez.argmax(), ez.shape)}"
        iu = np.triu_indices(b)
        Sd_ref = ref["S_diag"][:, iu[0], iu[1]].T
        scale = np.sqrt(np.abs(np.einsum("nii->ni", ref["S_diag"])))     # sqrt(S_ii)
        sc = (scale[:, iu[0]] * scale[:, iu[1]]).T
        es = np.abs(got["S_diag"] - Sd_ref) / sc
        assert es.max() <= tol, f"S_diag {es.max():.3e}"
        n = t.shape[0]
        if n > 1:
            Ss_ref = ref["S_sub"].reshape(n - 1, b * b).T
            rows = np.repeat(np.arange(b), b)
            cols = np.tile(np.arange(b), b)
            sc2 = scale[1:, rows].T * scale[:-1, cols].T
            eb = np.abs(got["S_sub"][:, : n - 1] - Ss_ref) / sc2
            assert eb.max() <= tol, f"S_sub {eb.max():.3e}"

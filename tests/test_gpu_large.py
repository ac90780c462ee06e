"""The large single series: Matern-5/2, N = 2^24, Exp(1) gaps.

Every output (logML with its two parts, gradient, posterior mean and latent variance at all
2^24 points) is compared with the C oracle.  The device memory the call needs is measured
against what storing every reduction level would take: only two tree elements per chunk of R
nodes are kept, the chunk-local levels are recomputed from (t, y) in the reverse sweep.
"""
import numpy as np
import pytest

from gpu_util import compare_series, to_dev
from workloads import make_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# bytes per node if every level of the reduction were stored: two elements per node (one per
# level on average) of A (9) + b (3) + Q (9) + J (9) + eta (3) doubles, at b = 3
EVERY_LEVEL_BYTES_PER_NODE = 2 * 33 * 8


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1610_08035_amd as spg
    spg.load_library()
    return spg


def test_config5_full_size(lib):
    w = make_config(5)
    t, y, hyp = w.series(0)
    n = t.shape[0]
    assert n == 1 << 24
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    h = lib.Handle(w.terms, n)
    td, yd, hd = to_dev(t), to_dev(y), to_dev(hyp)
    h.assemble(td, yd, hd)
    ll2, g = h.logml_grad()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    h.factor()
    ll, fit, ld = h.logml(parts=True)
    fm = h.solve()
    fv = h.selinv()
    rc, bad = h.status()
    got = {"logml": ll.item(), "datafit": fit.item(), "logdet": ld.item(), "logml2": ll2.item(),
           "grad": g.cpu().numpy().reshape(-1), "status": rc, "f_mean": fm.cpu().numpy(),
           "f_var": fv.cpu().numpy()}
    ws = h.workspace_bytes()
    h.close()
    compare_series(w.terms, t, y, hyp, got, blocks=False)
    # device memory of logML + gradient: inputs, workspace, outputs (and allocator slack)
    used = free0 - free1
    print(f"\nN = 2^24: library workspace {ws / 2**20:.1f} MiB, device memory of the call "
          f"{used / 2**20:.1f} MiB, every level stored {EVERY_LEVEL_BYTES_PER_NODE * n / 2**20:.1f} MiB")
    assert ws < 0.5 * EVERY_LEVEL_BYTES_PER_NODE * n
    # the logML + gradient workspace at 2^24 stays under 1 GB (the prediction buffers are
    # allocated only by spingp_predict)
    assert ws <= 1_000_000_000
    assert used < ws + 2 * 16 * n + (256 << 20)

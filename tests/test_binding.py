"""Host-side logic of the Python binding (no GPU, no library calls)."""
import torch

from paper_2201_08110_amd.nnp import NNP


def _fake():
    n = NNP.__new__(NNP)
    n.uploads = []
    n.set_weights = lambda w: n.uploads.append(w.copy())
    return n


def test_sync_params_uploads_only_on_change():
    n = _fake()
    p = torch.arange(6, dtype=torch.float64)
    n.sync_params(p)
    n.sync_params(p)
    assert len(n.uploads) == 1
    with torch.no_grad():
        p.add_(1.0)
    n.sync_params(p)
    assert len(n.uploads) == 2 and n.uploads[-1][0] == 1.0
    # a different tensor is always uploaded, even with equal contents and
    # even if it were to reuse the storage of a freed one
    for k in range(5):
        q = torch.full((6,), float(k), dtype=torch.float64)
        n.sync_params(q)
        assert n.uploads[-1][0] == float(k)
    assert len(n.uploads) == 7

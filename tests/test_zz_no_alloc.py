"""The allocation-free weight gradient (cnn_wgrad_noalloc, a file-scope device array as its
workspace) against cnn_wgrad with a caller workspace: identical results on two calls in a
row, the second smaller, and a clear error beyond the array's size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _inputs(rng, B, H, W, cin, cout):
    from paper_1111_0983_amd import cnn
    x = np.zeros((B, H, W, cnn.cpad(cin)), np.float32)
    x[..., :cin] = rng.normal(size=(B, H, W, cin))
    dy = np.zeros((B, H, W, cnn.cpad(cout)), np.float32)
    dy[..., :cout] = rng.normal(size=(B, H, W, cout))
    xt = torch.from_numpy(x).to(torch.bfloat16).to(DEV).reshape(-1)
    dyt = torch.from_numpy(dy).to(torch.bfloat16).to(DEV).reshape(-1)
    return xt, dyt


@pytest.mark.parametrize("cin,cout,dil", [(32, 32, 2), (4, 32, 1), (32, 1, 1)])
def test_noalloc_wgrad_matches_workspace_version(cin, cout, dil):
    from paper_1111_0983_amd import cnn
    rng = np.random.default_rng(cin * 100 + cout + dil)
    # a large call, then a smaller one: the second must not see the first one's partials
    for B, H, W in ((16, 65, 65), (3, 17, 29)):
        x, dy = _inputs(rng, B, H, W, cin, cout)
        dw_ref, db_ref = cnn.wgrad(x, dy, B, H, W, cin, cout, dil)
        dw = torch.full_like(dw_ref, float("nan"))
        db = torch.full_like(db_ref, float("nan"))
        cnn.wgrad_noalloc(x, dy, B, H, W, cin, cout, dil, dw, db)
        torch.cuda.synchronize()
        # the same kernels on the same inputs in the same order: bit-identical
        assert torch.equal(dw, dw_ref), (B, H, W)
        assert torch.equal(db, db_ref), (B, H, W)


def test_noalloc_wgrad_rejects_oversize():
    from paper_1111_0983_amd import cnn
    from paper_1111_0983_amd import ghostmg as gm
    B, H, W, cin, cout = 1, 1, 1, 32, 32
    x, dy = _inputs(np.random.default_rng(0), B, H, W, cin, cout)
    dw = torch.empty(cout * 9 * cin, dtype=torch.float32, device=DEV)
    db = torch.empty(cout, dtype=torch.float32, device=DEV)
    # 1024 x 1024 pixels need 1024 blocks of 9,248 partial sums: beyond the 4 Mi-float array
    # (the size check comes before any launch, so no kernel reads x or dy)
    with pytest.raises(gm.GhostMGError):
        cnn.wgrad_noalloc(x, dy, 1, 1024, 1024, cin, cout, 1, dw, db)

"""gs_l1_loss_static (no allocation, static device scratch) against
gs_l1_loss (caller scratch) through the C ABI: loss bit for bit and gradient
bit for bit (the same kernels and summation order), on two calls in a row,
the second with a smaller input, so the static array keeps the first call's
partial sums when the second runs."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2510_14564_amd import gs as mod
    return mod


def _pair(count, seed):
    rng = np.random.default_rng(seed)
    img = torch.from_numpy(rng.random(count, dtype=np.float32)).to(DEV)
    tgt = torch.from_numpy(rng.random(count, dtype=np.float32)).to(DEV)
    return img, tgt


def test_l1_loss_static_matches_caller_scratch(gs):
    # 1600x1064x3 floats (the main frame: 1024 partial sums), then a small
    # ragged count (3 partial sums) and a count below one workgroup
    for count, seed in ((3 * 1600 * 1064, 11), (513, 12), (37, 13)):
        print(f"[no-alloc l1] count={count}", flush=True)
        img, tgt = _pair(count, seed)
        loss_a = torch.empty(1, device=DEV)
        grad_a = torch.empty(count, device=DEV)
        partials = torch.empty(gs.L1_PARTIALS, device=DEV)
        gs.l1_loss(img, tgt, loss_a, grad_a, partials)
        loss_b = torch.full((1,), float("nan"), device=DEV)
        grad_b = torch.full((count,), float("nan"), device=DEV)
        gs.l1_loss_static(img, tgt, loss_b, grad_b)
        torch.cuda.synchronize()
        assert torch.equal(loss_a, loss_b), (loss_a.item(), loss_b.item())
        assert torch.equal(grad_a, grad_b)
        want = np.abs(img.cpu().numpy().astype(np.float64) - tgt.cpu().numpy()).mean()
        assert abs(loss_b.item() - want) <= 1e-5 * want


def test_l1_loss_static_without_gradient(gs):
    img, tgt = _pair(4096, 21)
    loss_a = torch.empty(1, device=DEV)
    loss_b = torch.empty(1, device=DEV)
    gs.l1_loss(img, tgt, loss_a, None, torch.empty(gs.L1_PARTIALS, device=DEV))
    gs.l1_loss_static(img, tgt, loss_b, None)
    torch.cuda.synchronize()
    assert torch.equal(loss_a, loss_b)


def test_l1_loss_static_rejects_bad_arguments(gs):
    img, tgt = _pair(16, 31)
    with pytest.raises(gs.GsError):
        gs.l1_loss_static(img[:0], tgt[:0], torch.empty(1, device=DEV), None)

"""sbli_mse_grad_noalloc (static device scratch, no allocation) against sbli_mse_grad
(caller workspace): same kernels, so bitwise the same gradient and loss, on two calls
in a row with the second one smaller (the scratch keeps the first call's partials)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_mse_grad_noalloc_matches_workspace_form():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    from paper_1609_01277_amd import closure
    rng = np.random.default_rng(2024)
    ms = torch.tensor([0.1, -0.2, 0.0, 0.05, 0.3, 0.8, 1.1, 0.9, 1.3, 0.7], device="cuda")
    for n, batch in ((64, 4), (32, 1)):
        P = n ** 3
        y = torch.from_numpy(rng.standard_normal((batch, P, 8)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.standard_normal((batch, 5, n, n, n)).astype(np.float32)).cuda()
        work = torch.empty(closure.sbli_mse_grad_work_bytes(n, batch) // 8, dtype=torch.float64, device="cuda")
        dy_ref = torch.empty((batch, P, 8), dtype=torch.bfloat16, device="cuda")
        loss_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        closure.sbli_mse_grad(y, 8, t, ms, n, batch, dy_ref, loss_ref, work)
        dy = torch.full((batch, P, 8), 7.0, dtype=torch.bfloat16, device="cuda")
        loss = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        closure.sbli_mse_grad_noalloc(y, 8, t, ms, n, batch, dy, loss)
        torch.cuda.synchronize()
        assert torch.equal(dy, dy_ref), (n, batch)
        assert loss.item() == loss_ref.item() and loss.item() > 0, (n, batch)


def test_mse_grad_noalloc_rejects_sizes_beyond_its_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a HIP device")
    from paper_1609_01277_amd import closure, _lib
    d = torch.zeros(8, device="cuda")
    with pytest.raises(_lib.SbliError) as ei:
        closure.sbli_mse_grad_noalloc(d, 8, d, d, 256, 2, d, d)    # 2 * 256^3 = 2^25 points
    assert ei.value.code == _lib.SBLI_ERR_ARG and "maximum" in str(ei.value)

"""The allocation-free gradient entry point (mc_lya_mlp_gradient_static, for
callers that cannot allocate device memory) against mc_lya_mlp_gradient, bit
for bit, on two calls in a row (the second on fewer cells, so that leftovers
of the first call in the shared static workspace would show), through the C
ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2312_11448_amd as M  # noqa: E402
from workloads import surrogate as WS  # noqa: E402


def _batch(rng, n):
    X = rng.normal(0.0, 1.0, size=(n, 8)).astype(np.float32)
    t = rng.normal(0.0, 0.3, size=n).astype(np.float32)
    w = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    w[::7] = 0.0
    return [torch.from_numpy(a).cuda() for a in (X, t, w)]


def test_static_gradient_equals_object_gradient():
    params = np.asarray(WS.initial_params(3), dtype=np.float32)
    rng = np.random.default_rng(11)
    d_params = torch.from_numpy(params.copy()).cuda()
    out = torch.full((M.MC_LYA_MLP_PARAMS + 2,), float("nan"), dtype=torch.float32, device="cuda")
    free_before = None
    for call, n in enumerate((150_000, 20_011)):
        X, t, w = _batch(rng, n)
        with M.Mlp(params) as mlp:
            g_ref, loss_ref = mlp.gradient(X, t, w)
        torch.cuda.synchronize()
        if call == 1:
            free_before = torch.cuda.mem_get_info()[0]
        M.mc_lya_mlp_gradient_static(d_params.data_ptr(), X.data_ptr(), t.data_ptr(), w.data_ptr(), n,
                                     out.data_ptr())
        torch.cuda.synchronize()
        if call == 1:
            assert torch.cuda.mem_get_info()[0] == free_before      # nothing allocated
        o = out.cpu().numpy()
        assert np.array_equal(o[:M.MC_LYA_MLP_PARAMS], np.asarray(g_ref, dtype=np.float32)), call
        loss = np.float32(o[M.MC_LYA_MLP_PARAMS]) / np.float32(o[M.MC_LYA_MLP_PARAMS + 1])
        assert loss == np.float32(loss_ref), call
        assert o[M.MC_LYA_MLP_PARAMS + 1] == pytest.approx(float(w.sum().item()), rel=1e-5)


def test_static_gradient_rejects_bad_sizes():
    X = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    v = torch.zeros(4, dtype=torch.float32, device="cuda")
    out = torch.zeros(M.MC_LYA_MLP_PARAMS + 2, dtype=torch.float32, device="cuda")
    p = torch.zeros(M.MC_LYA_MLP_PARAMS, dtype=torch.float32, device="cuda")
    for n in (0, M.MC_LYA_STATIC_MAX_CELLS + 1):
        with pytest.raises(M.MCLyaError) as e:
            M.mc_lya_mlp_gradient_static(p.data_ptr(), X.data_ptr(), v.data_ptr(), v.data_ptr(), n, out.data_ptr())
        assert e.value.status == M.MC_LYA_EINVAL
    with pytest.raises(M.MCLyaError) as e:
        M.mc_lya_mlp_gradient_static(p.data_ptr(), X.data_ptr(), v.data_ptr(), v.data_ptr(), 4, None)
    assert e.value.status == M.MC_LYA_EINVAL and "NULL" in str(e.value)

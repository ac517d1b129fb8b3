"""accord_prox_noalloc (the allocation-free prox) against accord_prox, through the C
ABI: the same kernels, so the same bits, on two calls in a row (the second smaller, so
it reuses the scratch array the first call left its partial sums in), and both against
the FP64 oracle's prox (eq. 3.5) at the bars of the prox parity test."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _case(p, seed):
    rng = np.random.default_rng(seed)
    om = np.where(rng.random((p, p)) < 0.3, rng.normal(0, 0.3, (p, p)), 0.0)
    om[np.diag_indices(p)] = rng.uniform(0.5, 2.0, p)
    g = rng.normal(0, 0.5, (p, p))
    return om.astype(np.float32), g.astype(np.float32)


def _noalloc(lib, om_t, g_t, tau, lam, out, red):
    """One call through the C ABI (argument marshalling only); returns the status."""
    import torch
    p = om_t.shape[0]
    return lib.accord_prox_noalloc(om_t.data_ptr(), g_t.data_ptr(), p, tau, lam, out.data_ptr(),
                                   red.data_ptr(), torch.cuda.current_stream().cuda_stream)


def test_prox_noalloc_matches_prox(gpu_lib):
    import torch
    lib = gpu_lib.lib()
    for p, tau, lam, seed in [(700, 0.37, 0.2, 1), (129, 0.125, 0.05, 2)]:
        print(f"[noalloc] p={p} tau={tau} lambda={lam}", flush=True)
        om32, g32 = _case(p, seed)
        om_t = torch.from_numpy(np.ascontiguousarray(om32.T)).cuda()   # column form
        g_t = torch.from_numpy(np.ascontiguousarray(g32.T)).cuda()
        ref_out, ref_red = gpu_lib.accord_prox(om_t, g_t, tau, lam)
        out = torch.empty_like(om_t)
        red = torch.empty(6, dtype=torch.float64, device="cuda")
        assert _noalloc(lib, om_t, g_t, tau, lam, out, red) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out)
        assert torch.equal(red, ref_red)
        # eq. 3.5 in FP64 on the same FP32 inputs
        got = out.cpu().numpy().T.astype(np.float64)
        o64, g64 = om32.astype(np.float64), g32.astype(np.float64)
        ref = oracle.prox(o64, g64, tau, lam)
        off = ~np.eye(p, dtype=bool)
        bound = 4 * U32 * (np.abs(o64) + tau * np.abs(g64) + tau * lam) + 1e-30
        assert np.all(np.abs(got - ref)[off] <= bound[off])
        d = np.diag_indices(p)
        assert np.all(np.abs(got[d] - ref[d]) <= np.spacing(np.abs(ref[d]).astype(np.float32)))
        dl = (got.astype(np.float32) - om32).astype(np.float64)
        r = red.cpu().numpy()
        assert np.isclose(r[0], np.sum(dl * dl), rtol=1e-12)
        assert r[4] == np.count_nonzero(got[off])


def test_prox_noalloc_rejects_bad_arguments(gpu_lib):
    import torch
    lib = gpu_lib.lib()
    om_t = torch.eye(16, device="cuda")
    g_t = torch.zeros(16, 16, device="cuda")
    red = torch.empty(6, dtype=torch.float64, device="cuda")
    assert _noalloc(lib, om_t, g_t, 0.0, 0.1, torch.empty_like(om_t), red) == 1   # tau
    assert _noalloc(lib, om_t, g_t, 0.5, 0.1, om_t, red) == 1                     # aliasing

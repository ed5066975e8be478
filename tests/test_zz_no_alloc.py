"""The allocation-free ALM-step entry point (lrsdp_k_alm_noalloc) against the
entry point with a caller work buffer (lrsdp_k_alm): the same multipliers and
measures, bit for bit, on two calls in a row where the second has a smaller
input (the static array keeps the first call's contents), for MaxCut and
completion in float64 and float32; sizes past the array are refused."""

import numpy as np
import pytest

from synth import chung_lu_edges, completion_instance, init_factor, pm1_weights

from paper_2407_15049_amd import lrsdp as L
from gpu_util import dev_factor, dev_vec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return L.Context(0)


def maxcut(n, seed):
    u, v = chung_lu_edges(n, 5 * n, 2.5, seed)
    return L.Problem.maxcut(n, u, v, pm1_weights(5 * n, seed + 1)), n


def completion(n1, n2, seed):
    i, j, Mij, _, _ = completion_instance(n1, n2, 4, 10, seed)
    return L.Problem.completion(n1, n2, i, j, Mij), len(i)


def compare(ctx, prob, m, prec, r, seed):
    import torch
    prob.upload(ctx)
    n = prob.info.n
    rng = np.random.default_rng(seed)
    R = dev_factor(init_factor(n, r, seed) * (1 + 0.05 * rng.standard_normal((n, 1))), prec)
    y0 = rng.standard_normal(m)
    ya, yb = dev_vec(y0), dev_vec(y0)
    oa = torch.zeros(8, dtype=torch.float64, device="cuda")
    ob = torch.zeros(8, dtype=torch.float64, device="cuda")
    work = torch.empty(8 * max(m, n * R.shape[1]), dtype=torch.uint8, device="cuda")
    L.k_alm(ctx, prob, prec, R, ya, 1.3, work, oa)
    L.k_alm_noalloc(ctx, prob, prec, R, yb, 1.3, ob)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    assert torch.equal(oa, ob)
    assert np.all(np.isfinite(ob.cpu().numpy()[:6]))


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_noalloc_maxcut_two_calls(ctx, prec):
    print("CASE", dict(test="noalloc_maxcut", prec=prec), flush=True)
    big, n_big = maxcut(150_000, 61)
    small, n_small = maxcut(9_001, 62)
    compare(ctx, big, n_big, prec, 20, 63)
    compare(ctx, small, n_small, prec, 12, 64)


@pytest.mark.parametrize("prec", [L.F64, L.F32])
def test_noalloc_completion_two_calls(ctx, prec):
    print("CASE", dict(test="noalloc_completion", prec=prec), flush=True)
    big, m_big = completion(40_000, 30_000, 65)
    small, m_small = completion(3_001, 2_000, 66)
    compare(ctx, big, m_big, prec, 16, 67)
    compare(ctx, small, m_small, prec, 8, 68)


def test_noalloc_refuses_sizes_past_the_array(ctx):
    import torch
    cap = L.k_alm_noalloc_max_bytes()
    assert cap == 64 << 20
    n = cap // (8 * 16) + 1                 # n x 16 float64 is one row past the array
    u = np.arange(n - 1, dtype=np.int32)
    prob = L.Problem.maxcut(n, u, u + 1).upload(ctx)
    R = torch.zeros((n, 16), dtype=torch.float64, device="cuda")
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LrsdpError) as e:
        L.k_alm_noalloc(ctx, prob, L.F64, R, y, 1.0, out)
    assert e.value.code == L.ENOMEM and "static" in str(e.value)

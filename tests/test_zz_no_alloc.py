"""pdn_surrogate_grad_noalloc (include/pdn.h), the gradient entry point that
allocates nothing, against the allocating pdn_surrogate_grad: same weights
and records, two calls in a row (the second smaller), bit-for-bit equal
gradient and loss; sizes beyond the fixed scratch are rejected."""
import sys

import numpy as np
import pytest
import torch

import paper_2301_05552_amd as pdn
import workloads as W

pytestmark = pytest.mark.gpu
EINVAL = -1


def _note(name):
    print(f"[gpu case] {name}", flush=True)
    sys.stdout.flush()


def _weights(seed):
    return W.rng(seed).uniform(-0.3, 0.3, pdn.SUR_NPARAM).astype(np.float32)


def _records(n, seed):
    g = W.rng(seed)
    x = g.standard_normal((n, 10)).astype(np.float32)
    t = (0.5 * g.standard_normal((n, 10))).astype(np.float32)
    return x, t


def test_noalloc_grad_equals_the_allocating_call():
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev).cuda_stream
    w = _weights(3)
    wd = torch.from_numpy(w).to(dev)
    for n, seed in ((3000, 11), (1000, 12), (pdn.SUR_GRAD_NOALLOC_MAX, 13)):
        _note(f"no-alloc grad n={n} seed={seed}")
        x, t = _records(n, seed)
        g_ref, l_ref = pdn.surrogate_grad(w, x, t, device=0, stream=stream)
        xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
        gd = torch.full((pdn.SUR_NPARAM,), float("nan"), dtype=torch.float32, device=dev)
        ld = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        pdn.surrogate_grad_noalloc(wd.data_ptr(), xd.data_ptr(), td.data_ptr(), n, gd.data_ptr(), ld.data_ptr(),
                                   device=0, stream=stream)
        torch.cuda.synchronize(dev)
        g = gd.cpu().numpy()
        assert np.isfinite(g).all()
        assert np.array_equal(g, g_ref), np.abs(g - g_ref).max()
        assert ld.item() == l_ref
    # loss pointer may be NULL
    gd.fill_(float("nan"))
    pdn.surrogate_grad_noalloc(wd.data_ptr(), xd.data_ptr(), td.data_ptr(), n, gd.data_ptr(), None,
                               device=0, stream=stream)
    torch.cuda.synchronize(dev)
    assert np.array_equal(gd.cpu().numpy(), g_ref)


def test_noalloc_grad_rejects_sizes_beyond_the_scratch():
    _note("no-alloc grad: size and argument errors")
    dev = torch.device("cuda:0")
    buf = torch.zeros(16, device=dev)
    p = buf.data_ptr()
    for n in (0, -3, pdn.SUR_GRAD_NOALLOC_MAX + 1):
        with pytest.raises(pdn.PdnError) as e:
            pdn.surrogate_grad_noalloc(p, p, p, n, p, None, device=0)
        assert e.value.code == EINVAL
        if n > 0:
            assert "exceed" in str(e.value)
    with pytest.raises(pdn.PdnError) as e:
        pdn.surrogate_grad_noalloc(p, None, p, 4, p, None, device=0)
    assert e.value.code == EINVAL

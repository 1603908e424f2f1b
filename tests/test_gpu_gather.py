"""GPU checks of gather_attrs and its hand-written backward against CPU
index_select autograd, gradcheck and finite differences."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _reindex(m):
    import paper_2109_09812_amd as mrx
    v = torch.from_numpy(np.ascontiguousarray(m.vtx).view(np.int32)).to(DEV)
    i = torch.from_numpy(m.idx).to(DEV)
    return mrx.reindex_mesh(v, i)


@pytest.mark.parametrize("channels,dtype,injective", [(16, torch.float32, False), (16, torch.float32, True),
                                                      (3, torch.float32, True), (16, torch.float64, False),
                                                      (5, torch.float64, True)])
def test_forward_backward_match_cpu_autograd(channels, dtype, injective):
    import paper_2109_09812_amd as mrx
    m = meshgen.grid_soup(200, 0.04, 17, "g")
    r = _reindex(m)
    n2o = r.new2old.cpu().numpy()
    assert np.array_equal(n2o, oracle.reindex(m.vtx, m.idx)[3])
    g = torch.Generator().manual_seed(channels)
    attrs = torch.randn(m.num_vtx, channels, generator=g, dtype=dtype)
    w = torch.randn(n2o.size, channels, generator=g, dtype=dtype)
    w[0, 0] = -0.0  # a negative zero gradient must land as +0.0, as accumulation into zeros gives
    _say("gather", channels, dtype, injective)
    a = attrs.to(DEV).requires_grad_(True)
    out = mrx.gather_attrs(a, r.new2old, injective=injective)
    (out * w.to(DEV)).sum().backward()
    ref = oracle.gather_attrs(attrs, n2o)
    ref_grad = oracle.gather_attrs_backward(w, n2o, m.num_vtx)
    assert torch.equal(out.detach().cpu(), ref)
    got = a.grad.cpu()
    assert torch.equal(got, ref_grad)
    assert torch.equal(torch.signbit(got), torch.signbit(ref_grad))
    # closed form: rows new2old[j] receive w[j], every other row is zero
    cf = torch.zeros_like(ref_grad)
    cf[torch.as_tensor(n2o, dtype=torch.long)] = 0 + w
    assert torch.equal(got, cf)


def test_non_injective_backward_accumulates():
    import paper_2109_09812_amd as mrx
    n2o = torch.tensor([3, 1, 3, 0, 3, 1], dtype=torch.int32)
    attrs = torch.arange(20, dtype=torch.float64).reshape(5, 4)
    g = torch.arange(24, dtype=torch.float64).reshape(6, 4) / 7
    _say("non-injective")
    a = attrs.to(DEV).requires_grad_(True)
    out = mrx.gather_attrs(a, n2o.to(DEV), injective=False)
    out.backward(g.to(DEV))
    ref = oracle.gather_attrs_backward(g, n2o.numpy(), 5)
    assert torch.allclose(a.grad.cpu(), ref, rtol=1e-12, atol=0)
    assert torch.equal(out.detach().cpu(), oracle.gather_attrs(attrs, n2o.numpy()))


def test_default_backward_is_safe_for_repeated_entries():
    """Without the injective promise the backward accumulates: a map with
    repeated entries gets every contribution (integer-valued gradients make
    each sum exact in any order)."""
    import paper_2109_09812_amd as mrx
    rng = np.random.default_rng(12)
    n2o = torch.from_numpy(rng.integers(0, 300, size=5000).astype(np.int32))
    attrs = torch.randn(300, 16, generator=torch.Generator().manual_seed(12))
    g = torch.from_numpy(rng.integers(-16, 17, size=(5000, 16)).astype(np.float32))
    _say("default backward, repeated entries")
    a = attrs.to(DEV).requires_grad_(True)
    mrx.gather_attrs(a, n2o.to(DEV)).backward(g.to(DEV))
    assert torch.equal(a.grad.cpu(), oracle.gather_attrs_backward(g, n2o.numpy(), 300))


def test_out_of_range_map_raises():
    import paper_2109_09812_amd as mrx
    a = torch.zeros(10, 4, device=DEV, requires_grad=True)
    _say("out-of-range map")
    for bad in ([0, 10, 2], [-1, 3]):
        with pytest.raises(IndexError):
            mrx.gather_attrs(a, torch.tensor(bad, dtype=torch.int32, device=DEV))
    # validate=False skips the check (documented): zero rows, no exception
    out = mrx.gather_attrs(a, torch.tensor([1, 10], dtype=torch.int32, device=DEV), validate=False)
    assert torch.equal(out[1].cpu(), torch.zeros(4))


def _submesh():
    big = meshgen.grid_soup(120, 0.04, 2109_09812 + 5, "soup")
    return meshgen.cfg5_submesh(big, 333)


def test_gradcheck_fp64_submesh():
    import paper_2109_09812_amd as mrx
    sub = _submesh()
    assert sub.num_vtx == 1000
    r = _reindex(sub)
    n2o = r.new2old
    attrs = torch.randn(sub.num_vtx, 4, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    a = attrs.to(DEV).requires_grad_(True)
    _say("gradcheck")
    assert torch.autograd.gradcheck(lambda x: mrx.gather_attrs(x, n2o), (a,), eps=1e-6, atol=1e-9)


def test_finite_differences_fp32_submesh():
    """loss = sum(w * gather(attrs)); central differences on sampled entries
    in fp32 (step 2^-4 on O(1) values: the loss is linear, so the difference
    quotient is exact up to the rounding of the two fp32 sums)."""
    import paper_2109_09812_amd as mrx
    sub = _submesh()
    r = _reindex(sub)
    n2o = r.new2old
    gen = torch.Generator().manual_seed(2)
    attrs = torch.randn(sub.num_vtx, 16, generator=gen)
    w = torch.randn(n2o.numel(), 16, generator=gen).to(DEV)
    a = attrs.to(DEV).requires_grad_(True)
    _say("finite differences")
    (mrx.gather_attrs(a, n2o) * w).sum().backward()
    grad = a.grad.cpu()
    h = 2.0 ** -4
    rng = np.random.default_rng(3)
    rows = rng.integers(0, sub.num_vtx, 60)
    cols = rng.integers(0, 16, 60)
    loss = lambda x: float((mrx.gather_attrs(x, n2o) * w).sum().double())
    base = attrs.to(DEV)
    scale = float(w.abs().sum())
    for i, c in zip(rows, cols):
        xp = base.clone(); xp[i, c] += h
        xm = base.clone(); xm[i, c] -= h
        fd = (loss(xp) - loss(xm)) / (2 * h)
        # fp32 summation of ~16k products: absolute error of each sum <= ~1e-6 * scale
        assert abs(fd - float(grad[i, c])) <= 1e-6 * scale / h + 1e-3, (i, c, fd, float(grad[i, c]))


def test_cfg5_gather_full_size():
    """The 10M-vertex soup with [10M, 16] fp32 features: forward and backward
    bitwise against CPU index_select autograd."""
    import paper_2109_09812_amd as mrx
    m = meshgen.cfg5_mesh()
    _say("soup10M gather")
    r = _reindex(m)
    n2o = r.new2old.cpu().numpy()
    assert n2o.size == 1251 * 1281
    attrs, w = meshgen.cfg5_features(m.num_vtx, n2o.size)
    a = attrs.to(DEV).requires_grad_(True)
    out = mrx.gather_attrs(a, r.new2old)
    (out * w.to(DEV)).sum().backward()
    assert torch.equal(out.detach().cpu(), oracle.gather_attrs(attrs, n2o))
    ref = torch.zeros_like(attrs)
    ref[torch.as_tensor(n2o, dtype=torch.long)] = 0 + w
    assert torch.equal(a.grad.cpu(), ref)

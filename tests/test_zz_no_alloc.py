"""The allocation-free query (lsnif_query_noalloc) against lsnif_query.

Both run the same kernels on the same rays; only where their workspace lives
differs, so the results must agree bit for bit.  Two calls in a row, the
second on a smaller batch, exercise the shared scratch array keeping the
first call's contents; a batch beyond the array's size is refused on the host.
"""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2504_21627_amd import lsnif
    return lsnif


def _bits(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_noalloc_matches_query(L, prec):
    import torch
    obj = W.configs.c1_object()
    big = W.sphere_to_box_rays(np.random.default_rng(11), 300_000, radius=2.0, half_box=1.0)
    small = W.configs.c1()["rays"][:3000]
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, prec, prec))
        results = []
        # allocation-free calls first, before the context has grown any workspace of its own
        for rays_np in (big, small):
            rays = torch.from_numpy(np.ascontiguousarray(rays_np, np.float32)).cuda()
            out = torch.full((len(rays_np), 6), -7.0, dtype=torch.float32, device="cuda")
            print(f"noalloc {prec}: {len(rays_np)} rays", flush=True)
            L.lsnif_query_noalloc(ctx, oid, rays, out)
            torch.cuda.synchronize()
            results.append((rays, out))
        for rays, out in results:
            ref = torch.empty_like(out)
            L.lsnif_query(ctx, oid, rays, ref)
            torch.cuda.synchronize()
            assert np.array_equal(_bits(out), _bits(ref)), len(rays)
            assert int((out[:, 0].view(torch.int32) == 1).sum()) > 0
    finally:
        L.lsnif_destroy(ctx)


def test_noalloc_refuses_oversize_batch(L):
    import torch
    obj = W.configs.c1_object()
    ctx = L.lsnif_create(0)
    try:
        oid = L.lsnif_build(ctx, L.ObjectDesc(obj, "fp16", "fp16"))
        n = L.NOALLOC_SCRATCH_BYTES // 40    # at least 45 bytes per ray (H = 18): too many
        rays = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
        out = torch.zeros((n, 6), dtype=torch.float32, device="cuda")
        with pytest.raises(L.LsnifError) as e:
            L.lsnif_query_noalloc(ctx, oid, rays, out)
        assert "allocation-free" in str(e.value)
        torch.cuda.synchronize()
        assert int(out.abs().sum()) == 0     # nothing was enqueued
        # the entry point still works after the refusal
        small = torch.from_numpy(np.ascontiguousarray(W.configs.c1()["rays"][:512], np.float32)).cuda()
        a, b = torch.empty((512, 6), device="cuda"), torch.empty((512, 6), device="cuda")
        L.lsnif_query_noalloc(ctx, oid, small, a)
        L.lsnif_query(ctx, oid, small, b)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(a), _bits(b))
    finally:
        L.lsnif_destroy(ctx)

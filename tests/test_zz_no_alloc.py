"""nmg_apply_fprime_noalloc, the BF16 filter F' with the library's fixed
device scratch for callers that cannot allocate, against the allocating entry
point nmg_apply_fprime with NMG_MIXED (same kernels, so bit-identical): on
consecutive calls that share the scratch, each smaller than the one before,
and with a clear rejection beyond the scratch limit."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_noalloc_fprime_matches_allocating_entry_point():
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    n, L, B = 255, 5, 64
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=2.56 / (n + 1), levels=L, max_batch=B, channels=(1, 32, 32, 1),
                                        ksize=3))
    g = torch.Generator().manual_seed(90)
    # full size first, then smaller inputs: fewer images, then coarser levels
    # (level 3 is 31^2, the single-workgroup filter that needs no scratch)
    for level, batch in ((0, 64), (0, 9), (1, 23), (3, 5)):
        m = h.level_size(level)
        print(f"case noalloc F' level {level} ({m}x{m}) batch {batch}", flush=True)
        x = (torch.randn(batch, m, m, generator=g) * 2.0).float().to(dev)
        ref = h.apply_fprime(level, x, "mixed")
        out = torch.full_like(x, float("nan"))
        h.apply_fprime_noalloc(level, x, out)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(out).all())
        assert torch.equal(out, ref), float((out - ref).abs().max())
    h.close()


def test_noalloc_fprime_limit():
    """511^2 needs 4 * batch * 512^2 bytes: batch 16 fills the 16 MiB scratch
    exactly and matches; batch 17 is rejected with a message naming the limit."""
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    n = 511
    h = nmg.setup_hierarchy(nmg.Problem(n=n, s=2.56 / (n + 1), levels=3, max_batch=17, channels=(1, 32, 32, 1),
                                        ksize=3))
    g = torch.Generator().manual_seed(91)
    print("case noalloc F' 511x511 batch 16 and 17", flush=True)
    x = torch.randn(17, n, n, generator=g).float().to(dev)
    ref = h.apply_fprime(0, x[:16].contiguous(), "mixed")
    out = torch.empty(16, n, n, dtype=torch.float32, device=dev)
    h.apply_fprime_noalloc(0, x[:16].contiguous(), out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    with pytest.raises(nmg.NMGError) as ei:
        h.apply_fprime_noalloc(0, x, torch.empty_like(x))
    assert ei.value.code == -2 and "limit" in str(ei.value)
    h.close()


def test_noalloc_fprime_rejects_1d():
    from paper_2603_01064_amd import nmg
    dev = torch.device("cuda:0")
    h = nmg.setup_hierarchy(nmg.Problem(n=63, s=0.02, levels=3, dim=1, max_batch=2, channels=(1, 8, 8, 1),
                                        ksize=5))
    x = torch.zeros(2, 63, dtype=torch.float32, device=dev)
    with pytest.raises(nmg.NMGError) as ei:
        h.apply_fprime_noalloc(0, x, torch.empty_like(x))
    assert ei.value.code == -1
    h.close()

"""Stream ordering of a context bound to caller memory (mmc_bind, through mmc.Workspace)."""
import pytest


@pytest.mark.gpu
def test_tuner_waits_for_work_queued_on_the_bound_stream():
    """The first run of a context tunes it, and the tuner's trial launches write the
    workspace. With caller memory bound, they must wait for the work already queued on the
    bound stream. Here torch frees a buffer whose last reader is still queued behind a long
    chain of kernels; the workspace takes the same block from torch's caching allocator; the
    queued reader must still see the buffer's own contents, not the tuner's spins."""
    import torch
    from paper_1305_6758_amd import mmc
    torch.cuda.set_device(0)
    # FP64 at L = 14: only the generic variants fit (several candidates, so the tuner launches)
    ctx = mmc.mmc_create_ex(14, 1.5, 1.0, 6, 4, 4, 1234, mmc.config(precision=mmc.MMC_FP64))
    try:
        size = max(mmc.mmc_workspace_bytes(ctx), 256) + 256  # what Workspace allocates
        x = torch.full((size,), 7, dtype=torch.uint8, device="cuda")
        ptr = x.data_ptr()
        a = torch.rand(4096, 4096, device="cuda")
        for _ in range(150):  # a few hundred milliseconds of queued work
            a = torch.tanh(a @ a)
        x.add_((a[0, 0] * 0).to(torch.uint8))  # x's last write waits for the chain
        total = x.sum(dtype=torch.int64)         # its reader, queued behind that
        del x, a
        ws = mmc.Workspace(ctx)
        if ws.buf.data_ptr() != ptr:
            pytest.skip("the caching allocator did not hand the freed block to the workspace")
        mmc.mmc_run(ctx)
        torch.cuda.synchronize()
        assert int(total) == 7 * size
        assert "any" in mmc.mmc_plan(ctx)
    finally:
        mmc.mmc_destroy(ctx)

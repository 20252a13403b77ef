"""dc_analyze_noalloc (the entry point that allocates nothing) against
dc_analyze_batch on the same records, byte for byte: two calls in a row, the
second on a smaller batch, so the shared scratch array holds the first
call's contents when the second runs."""
import numpy as np
import pytest

import dcgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402


def say(*a):
    print(*a, flush=True)


def dev_bytes(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).reshape(-1).copy()).cuda()


def noalloc_run(ctx, b, flags):
    K, N = b.n_kernels, b.n_instr
    kdev, idev, adev = dev_bytes(b.kernels), dev_bytes(b.instrs), dev_bytes(b.args)
    res = torch.zeros(K * dc.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    acc = torch.zeros(N * dc.ACCESS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    sysv = torch.zeros(4 * N * dc.SYSVAL_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    aoff = torch.zeros(K + 1, dtype=torch.int32, device="cuda")
    soff = torch.zeros(K + 1, dtype=torch.int32, device="cuda")
    ctx.analyze_noalloc(kdev, K, N, idev, N, adev, len(b.args), res, acc, N, aoff, sysv, 4 * N, soff, flags=flags)
    torch.cuda.synchronize()
    r = res.cpu().numpy().view(dc.RESULT_DTYPE)
    ao = aoff.cpu().numpy().view(np.uint32)
    so = soff.cpu().numpy().view(np.uint32)
    a = acc.cpu().numpy().view(dc.ACCESS_DTYPE)[:ao[K]]
    s = sysv.cpu().numpy().view(dc.SYSVAL_DTYPE)[:so[K]]
    return r, a, s, ao, so


def batch_run(ctx, b, flags):
    dev = dc.to_device(b.instrs)
    bt = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=flags)
    r = bt.results()
    a, ao = bt.all_accesses()
    s, so = bt.all_sysvals()
    bt.free()
    return r, a, s, ao, so


def test_noalloc_matches_batch_twice():
    ctx = dc.Context(0)
    big = dcgen.generate(2, 240, i0=11)
    small = dcgen.generate(3, 60, i0=500)
    assert big.n_instr <= dc.NOALLOC_MAX_INSTR and small.n_instr < big.n_instr
    for name, b in (("first, larger", big), ("second, smaller", small)):
        say(f"noalloc: {name}: {b.n_kernels} kernels, {b.n_instr} instructions")
        for flags in (dc.OPT_DIGEST, 0):
            got = noalloc_run(ctx, b, flags)
            want = batch_run(ctx, b, flags)
            assert (want[0]["status"] == 0).all()
            assert got[0].tobytes() == want[0].tobytes(), name
            assert got[1].tobytes() == want[1].tobytes(), name
            assert got[2].tobytes() == want[2].tobytes(), name
            assert np.array_equal(got[3], want[3].astype(np.uint32)) and np.array_equal(got[4], want[4].astype(np.uint32))
    ctx.close()


def test_noalloc_limits_and_bad_totals():
    """Sizes past the limits are rejected before anything is enqueued; a
    wrong instruction total fails every kernel with DC_E_INVAL."""
    ctx = dc.Context(0)
    b = dcgen.generate(1, 8)
    K, N = b.n_kernels, b.n_instr
    kdev, idev, adev = dev_bytes(b.kernels), dev_bytes(b.instrs), dev_bytes(b.args)
    res = torch.zeros(K * 32, dtype=torch.uint8, device="cuda")
    acc = torch.zeros(N * 16, dtype=torch.uint8, device="cuda")
    sysv = torch.zeros(4 * N * 8, dtype=torch.uint8, device="cuda")
    aoff = torch.zeros(K + 1, dtype=torch.int32, device="cuda")
    soff = torch.zeros(K + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(dc.DCError) as e:
        ctx.analyze_noalloc(kdev, K, dc.NOALLOC_MAX_INSTR + 1, idev, N, adev, len(b.args), res, acc, N, aoff, sysv,
                            4 * N, soff)
    assert e.value.code == -1
    with pytest.raises(dc.DCError):
        ctx.analyze_noalloc(kdev, dc.NOALLOC_MAX_KERNELS + 1, N, idev, N, adev, len(b.args), res, acc, N, aoff,
                            sysv, 4 * N, soff)
    ctx.analyze_noalloc(kdev, K, N - 1, idev, N, adev, len(b.args), res, acc, N, aoff, sysv, 4 * N, soff)
    torch.cuda.synchronize()
    r = res.cpu().numpy().view(dc.RESULT_DTYPE)
    assert (r["status"] == -1).all() and int(aoff.cpu()[K]) == 0
    ctx.close()

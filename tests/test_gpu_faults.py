"""Device allocation failures (DC_FAULT_ALLOC=n makes the n-th device
allocation of each allocation list fail): every entry point that allocates
returns DC_E_OOM cleanly for every n, or succeeds with correct results, and
the library works normally afterwards."""
import numpy as np
import pytest

import dcgen
import oracle
from gpu_common import compare_ssa_summaries, compare_struct_summaries, compare_summaries, compare_types_summaries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402

OOM = -3


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch():
    b = dcgen.concat([dcgen.generate(2, 48, i0=77).kernel(k) for k in range(48)] +
                     [dcgen.generate(6, 12).kernel(9)])   # one kernel over 2,048 blocks: the overflow pass
    return b, dc.to_device(b.instrs)


def sweep(monkeypatch, call, check, n_max=80):
    """call() under DC_FAULT_ALLOC = 1..n_max: each either raises DC_E_OOM or
    returns an object that check() accepts; returns how many failed."""
    failed = 0
    for n in range(1, n_max + 1):
        monkeypatch.setenv("DC_FAULT_ALLOC", str(n))
        try:
            obj = call()
        except dc.DCError as e:
            assert e.code == OOM, (n, e)
            failed += 1
            continue
        finally:
            monkeypatch.delenv("DC_FAULT_ALLOC", raising=False)
        check(obj)
        obj.free()
    return failed


def test_analyze_batch_allocation_failures(ctx, batch, monkeypatch):
    b, dev = batch
    s, oacc, osys = oracle.analyze_batch(b)

    def check(bt):
        compare_summaries(bt.results(), s)
        assert bt.all_accesses()[0].tobytes() == oacc.tobytes()
    assert sweep(monkeypatch, lambda: ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST),
                 check) >= 10
    bt = ctx.analyze(b.kernels, dev, b.n_instr, b.args, flags=dc.OPT_DIGEST)
    check(bt)
    bt.free()


def test_versions_and_text_allocation_failures(ctx, batch, monkeypatch):
    b, dev = batch
    ss = oracle.ssa_batch(b)
    assert sweep(monkeypatch, lambda: ctx.build_ssa(b.kernels, dev, b.n_instr),
                 lambda s: compare_ssa_summaries(s.results(), ss)) >= 5
    text = dcgen.render(b)
    tdev = dc.text_to_device(text)
    o = oracle.parse_text(text)
    assert sweep(monkeypatch, lambda: ctx.parse_text(tdev, len(text)),
                 lambda t: (t.records().tobytes() == o["instrs"].tobytes()) or pytest.fail("records")) >= 5


def test_types_and_structuring_allocation_failures(ctx, batch, monkeypatch):
    b, dev = batch
    ts = oracle.types_batch(b)
    assert sweep(monkeypatch, lambda: ctx.build_types(b.kernels, dev, b.n_instr, b.args),
                 lambda t: compare_types_summaries(t.types(), ts)) >= 5
    st = oracle.structure_batch(b)
    assert sweep(monkeypatch, lambda: ctx.structure(b.kernels, dev, b.n_instr),
                 lambda x: compare_struct_summaries(x.results(), st)) >= 3


def test_server_allocation_failures(ctx, batch, monkeypatch):
    """A server whose lanes cannot be allocated is not created (DC_E_OOM);
    one that is created serves correctly."""
    b, _ = batch
    s, _, _ = oracle.analyze_batch(b)
    reqs = dc.requests(b.kernels, b.instrs, b.args)

    def check(srv):
        for i in range(len(reqs)):
            srv.submit(reqs, i)
        got = {}
        import time
        t0 = time.time()
        while len(got) < len(reqs) and time.time() - t0 < 60:
            for r in srv.poll(records=False)[0]:
                got[int(r["tag"])] = r
        assert len(got) == len(reqs)
        for i in range(len(reqs)):
            assert got[i]["summary"]["status"] == s[i]["status"] and got[i]["summary"]["n_blocks"] == s[i]["n_blocks"]

    class Srv:
        def __init__(self):
            self.s = dc.Server(ctx, lanes=2, max_request_instr=16384)

        def submit(self, reqs, i):
            return self.s.submit(reqs, i)

        def poll(self, **kw):
            return self.s.poll(**kw)

        def results(self):
            return None

        def free(self):
            self.s.close()
    assert sweep(monkeypatch, Srv, check, n_max=40) >= 5

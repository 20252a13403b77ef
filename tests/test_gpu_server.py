"""GPU parity of the request server (dc_server_*): continuous batching.

Requests arrive one at a time while earlier ones are on the device; every
result must equal the oracle's for that kernel alone (bit-exact), whatever
it was batched with, and batches must actually overlap on the device."""
import time

import numpy as np
import pytest

import dcgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


DRAIN_SECONDS = 120.0


def drain(srv, want, got, timeout=None):
    timeout = DRAIN_SECONDS if timeout is None else timeout
    t0 = time.time()
    while len(got) < want:
        res, recs = srv.poll()
        for r, rc in zip(res, recs):
            got[int(r["tag"])] = (r, rc)
        if time.time() - t0 > timeout:
            raise AssertionError(f"only {len(got)} of {want} results after {timeout} s: {srv.stats()}")
        if not len(res):
            time.sleep(0.0005)
    return got


def submit_poisson(srv, reqs, rate, seed, got):
    """Submit every request at Poisson arrival times (rate per second),
    polling between arrivals."""
    rng = np.random.default_rng(seed)
    due = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
    t0 = time.perf_counter()
    i = 0
    while i < len(reqs):
        now = time.perf_counter() - t0
        while i < len(reqs) and due[i] <= now:
            srv.submit(reqs, i)
            i += 1
        res, recs = srv.poll()
        for r, rc in zip(res, recs):
            got[int(r["tag"])] = (r, rc)


def oracle_split(b):
    summ, acc, sysv = oracle.analyze_batch(b)
    ao = np.zeros(len(summ) + 1, np.int64)
    so = np.zeros(len(summ) + 1, np.int64)
    ao[1:] = np.cumsum(summ["n_acc"])
    so[1:] = np.cumsum(summ["n_sys"])
    return [(summ[k], acc[ao[k]:ao[k + 1]], sysv[so[k]:so[k + 1]]) for k in range(len(summ))]


def check_against_oracle(got, ref, digest=True):
    for k, (s, oacc, osys) in enumerate(ref):
        r, (acc, sysv) = got[k]
        g = r["summary"]
        assert (g["status"], g["n_blocks"], g["sweeps"], g["n_access"], g["n_sysval"]) == \
            (s["status"], s["n_blocks"], s["sweeps"], s["n_acc"], s["n_sys"]), (k, g, s)
        if digest:
            assert g["digest"] == s["digest"], k
        assert acc.tobytes() == oacc.tobytes(), k
        assert sysv.tobytes() == osys.tobytes(), k
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_enqueued_ns"] <= r["t_device_ns"] <= r["t_done_ns"], k


def same_result(a, b):
    (ra, (aa, sa)), (rb, (ab, sb)) = a, b
    return ra["summary"].tobytes() == rb["summary"].tobytes() and aa.tobytes() == ab.tobytes() and \
        sa.tobytes() == sb.tobytes()


def test_server_stream_matches_oracle_alone_and_in_the_mix(ctx):
    """3,000 log-normal requests (median 1,000 instructions, cap 100k) at
    Poisson arrivals: every result equals the oracle's; batches overlap on
    the device; a sample of requests run alone give byte-identical results."""
    n = 3000
    b = dcgen.generate(5, n)
    say("server: generated", b.n_instr)
    ref = oracle_split(b)
    say("server: oracle done")
    reqs = dc.requests(b.kernels, b.instrs, b.args)
    srv = dc.Server(ctx, lanes=4, flags=dc.OPT_DIGEST)
    try:
        alone = {}
        sample = [int(x) for x in np.random.default_rng(5).choice(n, 12, replace=False)]
        for k in sample:
            srv.submit(reqs, k)
            one = drain(srv, 1, {})
            alone[k] = one[k]
            assert one[k][0]["batch_kernels"] == 1
        say("server: alone runs done")
        got = {}
        submit_poisson(srv, reqs, rate=20000.0, seed=11, got=got)
        drain(srv, n, got)
        st = srv.stats()
        say("server: mix done", st)
    finally:
        srv.close()
    check_against_oracle(got, ref)
    for k in sample:
        assert same_result(alone[k], got[k]), k
    # continuous batching: more than one request per batch somewhere, and two
    # batches in flight at the same time
    res = np.array([got[k][0] for k in range(n)])
    assert res["batch_kernels"].max() > 1
    spans = {}
    for r in res:
        a, d = spans.get(int(r["batch"]), (r["t_admit_ns"], r["t_done_ns"]))
        spans[int(r["batch"])] = (min(a, r["t_admit_ns"]), max(d, r["t_done_ns"]))
    iv = sorted(spans.values())
    overlap = any(iv[i + 1][0] < iv[i][1] for i in range(len(iv) - 1))
    assert overlap, "no two batches were in flight together"
    lat = (res["t_done_ns"] - res["t_submit_ns"]) / 1e6
    say(f"server: latency p50 {np.percentile(lat, 50):.2f} ms p99 {np.percentile(lat, 99):.2f} ms, "
        f"{len(spans)} batches, largest {res['batch_kernels'].max()}")


def test_server_bad_requests_fail_alone(ctx):
    """Malformed requests get their own status and leave their batch-mates
    exact; a request longer than the server accepts is refused at submit."""
    good = dcgen.generate(2, 6, i0=900)
    parts = [good.kernel(k) for k in range(6)]
    r, d, a = good.kernel(0)
    bad_op = r.copy()
    bad_op[3]["op"] = 200
    d_noargs = d.copy()
    d_noargs["useargs"] = 0
    d_many = d.copy()
    d_many["n_args"] = 300
    empty_d = d.copy()
    parts += [(bad_op, d, a), (r, d_noargs, a), (r, d_many, np.zeros(0, a.dtype)), (r[:0], empty_d, a)]
    b = dcgen.concat(parts)
    b.kernels["n_args"][8] = 300   # concat recounts n_args from the table
    ref = oracle_split(b)
    srv = dc.Server(ctx, lanes=2, max_request_instr=4000, flags=dc.OPT_DIGEST)
    try:
        reqs = dc.requests(b.kernels, b.instrs, b.args)
        got = {}
        for k in range(b.n_kernels):
            srv.submit(reqs, k)
        drain(srv, b.n_kernels, got)
        long_b = dcgen.concat([(np.zeros(4001, dcgen.INSTR_DTYPE), dcgen.descriptor(4001), a)])
        with pytest.raises(dc.DCError) as e:
            srv.submit(dc.requests(long_b.kernels, long_b.instrs, long_b.args), 0)
        assert e.value.code == -1
    finally:
        srv.close()
    statuses = [int(got[k][0]["summary"]["status"]) for k in range(b.n_kernels)]
    assert statuses[6:] == [-10, -14, -14, -13], statuses
    check_against_oracle(got, ref)


def test_server_long_and_dense_requests(ctx):
    """Long Zipf requests and dense-CFG requests (up to 2,500 blocks, taking
    the overflow pass inside a lane), each batch holding one length class."""
    z = dcgen.generate(3, 400, i0=20000)
    long_idx = np.nonzero(z.kernels["n_instr"] >= 4000)[0][:30]
    short_idx = np.nonzero(z.kernels["n_instr"] < 4000)[0][:200]
    dense = dcgen.generate(6, 8)
    parts = [z.kernel(int(k)) for k in long_idx] + [z.kernel(int(k)) for k in short_idx] + \
        [dense.kernel(k) for k in range(8)]
    order = np.random.default_rng(3).permutation(len(parts))
    b = dcgen.concat([parts[i] for i in order])
    ref = oracle_split(b)
    srv = dc.Server(ctx, lanes=3, long_instr=4000, flags=dc.OPT_DIGEST)
    try:
        reqs = dc.requests(b.kernels, b.instrs, b.args)
        got = {}
        submit_poisson(srv, reqs, rate=5000.0, seed=4, got=got)
        drain(srv, b.n_kernels, got)
    finally:
        srv.close()
    check_against_oracle(got, ref)
    assert max(int(s["n_blocks"]) for s, _, _ in ref) > 2048
    # a batch holds requests of one length class (bounds 250, 1000, 4000)
    by_batch = {}
    for k in range(b.n_kernels):
        r = got[k][0]
        cls = int(np.searchsorted([250, 1000, 4000], int(b.kernels["n_instr"][k]), side="right"))
        by_batch.setdefault(int(r["batch"]), set()).add(cls)
    assert all(len(v) == 1 for v in by_batch.values())

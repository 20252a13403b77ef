"""GPU parity of the structuring (Section "Search for control structures"):
the HIP search through the C ABI (dc_structure) against the oracle,
bit-exact on every merge, the regions left and the root; at full size
through the per-kernel digest over the merges."""
import sys

import numpy as np
import pytest

import asmtext
import dcgen
import hand_kernels as hk
import oracle
from gpu_common import OracleStructRun, compare_struct_summaries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2107_07809_amd import dc  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = dc.Context(0)
    yield c
    c.close()


def full_compare(ctx, b, label):
    say(f"struct {label}: {b.n_kernels} kernels, {b.n_instr} instructions")
    dev = dc.to_device(b.instrs)
    s = ctx.structure(b.kernels, dev, b.n_instr)
    res = s.results()
    for k in range(b.n_kernels):
        recs, d, _ = b.kernel(k)
        o = oracle.structure(recs, d)
        g = res[k]
        assert (g["status"], g["n_blocks"], g["n_left"], g["root"]) == (o["status"], o["n_blocks"], o["n_left"],
                                                                       o["root"]), k
        m = s.merges(k)
        assert m.tobytes() == o["merges"].tobytes(), (k, m[:4], o["merges"][:4])
        assert g["digest"] == o["digest"] and g["n_merges"] == len(o["merges"]), k
    s.free()
    return res


def test_paper_trace_and_templates(ctx):
    """The Fig. 3 trace and every hand-written template case of the oracle's
    pins, one kernel each, in one batch."""
    import test_oracle_structure as T
    srcs = [T.FIG3]
    for fn in (T.test_if_else_standard_form, T.test_exec_mask_if_else_reduces_as_two_ifs, T.test_loops,
               T.test_search_order_is_preorder_fall_through_first, T.test_irreducible_graph_stays_unreduced,
               T.test_unreachable_blocks_take_no_part, T.test_if_on_the_taken_edge,
               T.test_entry_is_never_an_inner_region, T.test_entry_is_not_a_loop_body):
        srcs += [c for c in fn.__code__.co_consts if isinstance(c, str) and "s_endpgm" in c]
    parts = []
    for src in srcs:
        recs = asmtext.assemble(src)
        parts.append((recs, dcgen.descriptor(len(recs)), np.zeros(0, dcgen.ARG_DTYPE)))
    assert len(parts) >= 12
    res = full_compare(ctx, dcgen.concat(parts), "templates")
    assert res[0]["n_merges"] == 4 and res[0]["root"] == 9


def test_generated_and_failing_kernels(ctx):
    """The small workload, log-uniform and Zipf samples, kernels of 1,500 to
    2,500 blocks (regions in global memory), the hand-written kernels and
    kernels that fail their checks, one batch."""
    good = dcgen.generate(2, 6)
    r, d, a = good.kernel(0)
    bad_op = r.copy()
    bad_op[5]["op"] = 200
    parts = [dcgen.generate(1, 32).kernel(k) for k in range(32)] + \
        [dcgen.generate(2, 300, i0=800).kernel(k) for k in range(300)] + \
        [dcgen.generate(3, 300, i0=31).kernel(k) for k in range(300)] + \
        [dcgen.generate(6, 12).kernel(k) for k in (0, 5, 9)] + \
        [k for _, k in hk.all_kernels()] + [(bad_op, d, a), (r[:-1].copy(), d, a)]
    res = full_compare(ctx, dcgen.concat(parts), "generated")
    assert (res["status"] < 0).sum() == 2 and (res["n_blocks"] > 1000).sum() >= 3


def test_c2_full_digest(ctx):
    """All 65,536 kernels of the log-uniform workload; a second run of the
    same object gives the same bytes."""
    n = 65536
    orc = OracleStructRun(2, n)
    b = dcgen.generate(2, n)
    dev = dc.to_device(b.instrs)
    s = ctx.structure(b.kernels, dev, b.n_instr)
    res = s.results()
    s.run()
    assert s.results().tobytes() == res.tobytes()
    s.free()
    compare_struct_summaries(res, orc.result())


def test_c3_zipf_full(ctx):
    """All 1,048,576 kernels of the Zipf(1.2) 20-20,000 workload (1.74e9
    instructions) in one object, against the oracle's summaries."""
    n = 1048576
    orc = OracleStructRun(3, n, jobs_per_proc=16)
    b = dcgen.generate(3, n)
    dev = dc.to_device(b.instrs)
    s = ctx.structure(b.kernels, dev, b.n_instr)
    res = s.results()
    s.free()
    del dev
    torch.cuda.empty_cache()
    compare_struct_summaries(res, orc.result())


def test_c4_very_large(ctx):
    """The 16 kernels of 1-4M instructions (up to ~17k blocks)."""
    orc = OracleStructRun(4, 16, procs=16, jobs_per_proc=1)
    b = dcgen.generate(4, 16)
    dev = dc.to_device(b.instrs)
    s = ctx.structure(b.kernels, dev, b.n_instr)
    res = s.results()
    s.free()
    say(f"struct c4: merges max {int(res['n_merges'].max())}")
    compare_struct_summaries(res, orc.result())

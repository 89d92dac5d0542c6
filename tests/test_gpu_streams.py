"""Calls on one context from alternating HIP streams.

Every call on a context shares its scratch (primitive buffers, stage states,
counters).  A caller that switches streams between calls must still see each
call ordered after the previous one: dg_set_stream makes the new stream wait
for the work queued on the old one.  Checked bit for bit against the same
calls on a single stream, with work queued behind long stage launches so that
an unordered stream would overlap them."""
import pytest
import torch

from paper_2205_00095_amd import workloads as wl

from ._util import oracle_state

pytestmark = pytest.mark.gpu


def _solver(cfg):
    from paper_2205_00095_amd.solver import Solver
    return Solver(cfg, sync=False)


def test_alternating_streams_match_single_stream():
    cfg = wl.make_config("kh_tm", n_elem=(64, 64, 1))
    st, U = oracle_state(cfg)
    dt = cfg["dt"]

    def sequence(s, streams):
        outs = []
        Ua = U.cuda().contiguous()
        Ub = U.cuda().contiguous()
        with torch.cuda.stream(streams[0]):
            s.run(Ua, dt, 20)                  # long run writing the shared stage buffers
        with torch.cuda.stream(streams[1]):
            Ub.copy_(U.cuda())
            R = s.rhs(Ub)                      # reuses the primitive scratch
            outs.append(R)
        with torch.cuda.stream(streams[0]):
            streams[0].wait_stream(streams[1])
            s.run(Ub, dt, 3)
        with torch.cuda.stream(streams[1]):
            streams[1].wait_stream(streams[0])
            R2 = s.rhs(Ua)
            outs.append(R2)
        torch.cuda.synchronize()
        return [Ua.cpu(), Ub.cpu()] + [o.cpu() for o in outs]

    ref_stream = torch.cuda.Stream()
    ref = sequence(_solver(cfg), [ref_stream, ref_stream])
    alt = sequence(_solver(cfg), [torch.cuda.Stream(), torch.cuda.Stream()])
    for a, b in zip(ref, alt):
        assert torch.equal(a.view(torch.int64), b.view(torch.int64))

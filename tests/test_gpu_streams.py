"""One context used from two torch streams in turn: switching the context's stream
waits for the work already queued on the previous one, whose buffers the next call
rewrites, so every call gives what it gives alone."""
import pytest
import workloads as W

pytestmark = pytest.mark.gpu


def test_calls_alternating_between_two_streams(lv_mod):
    import torch
    lv = lv_mod
    wl = W.small_call()
    s, b = wl.surface, wl.book
    sig = torch.tensor(s.sigma, dtype=torch.float64, device="cuda")
    ctx = lv.Context(0)

    def call(n_paths, n_steps):
        return lv.price_and_grad_dev(sig, 100.0, b.strike, b.maturity, n_paths, n_steps, wl.seed,
                                     spot_axis=s.spot_axis, time_axis=s.time_axis, adjoint="stored", ctx=ctx)

    # two requests of different sizes: the second rewrites the tables and the states
    req = [(1 << 19, 156), (1 << 17, 52)]
    refs = [[t.cpu() for t in call(*r)] for r in req]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        outs = []
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                outs.append(call(*req[k]))
        torch.cuda.synchronize()
        for k in range(2):
            for x, y in zip(outs[k], refs[k]):
                assert torch.equal(x.cpu(), y), (rep, k)


@pytest.fixture(scope="module")
def lv_mod():
    import paper_2002_02481_amd as m
    return m

"""The fused path inside a HIP graph: sal_saliency with a caller workspace allocates and
synchronises nothing, so it can be captured once and replayed.  Every replay (with eager
work and synchronisations between replays, and new data copied into the captured input)
must equal the eager call bit for bit."""
import pytest
import torch

from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,prec,stride", [(8, sal.FP32, 1), (16, sal.BF16_SPLIT, 1), (5, sal.FP32, 1),
                                           (8, sal.FP32, 2), (16, sal.FP32, 1), (16, sal.FP32, 4)])
def test_graph_replay_matches_eager(L, prec, stride):
    shape = (40, 48, 56)
    ctx = sal.Saliency(L=L, precision=prec, stride=stride)
    vols = [torch.from_numpy(synth.make_volume(shape, seed=s, n_faults=1, n_chaotic=1, chaotic_size=12)).cuda()
            for s in (1, 2, 3)]
    V = vols[0].clone()
    S = torch.empty_like(V)
    Sr = torch.empty((3,) + shape, dtype=torch.float32, device="cuda")
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = ctx.workspace(shape)
    ctx.saliency(V, S=S, S_raw_out=Sr, stats_out=st, workspace=ws)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.saliency(V, S=S, S_raw_out=Sr, stats_out=st, workspace=ws)
    for rep, src in enumerate(vols + vols[:1]):
        V.copy_(src)
        g.replay()
        torch.cuda.synchronize()
        got = (S.clone(), Sr.clone(), st.clone())
        # eager reference on separate buffers, with other work in between
        _ = (src * 2.0).sum().item()
        S_e = torch.empty_like(V)
        Sr_e = torch.empty_like(Sr)
        st_e = torch.zeros_like(st)
        ctx.saliency(src, S=S_e, S_raw_out=Sr_e, stats_out=st_e)
        torch.cuda.synchronize()
        assert torch.equal(got[0], S_e), rep
        assert torch.equal(got[1], Sr_e), rep
        assert torch.equal(got[2][:7], st_e[:7]), rep


def test_two_contexts_on_two_streams():
    """Two contexts driven concurrently from two streams (each call on its caller's stream,
    no hidden device-wide synchronisation or shared state) give exactly the results each
    gives alone."""
    shape = (36, 40, 52)
    V1 = torch.from_numpy(synth.make_volume(shape, seed=4, n_faults=1)).cuda()
    V2 = torch.from_numpy(synth.make_volume(shape, seed=5, n_faults=2)).cuda()
    c1 = sal.Saliency(L=8)
    c2 = sal.Saliency(L=16, precision=sal.BF16_SPLIT)
    ref1 = c1.saliency_maps(V1)
    ref2 = c2.saliency_maps(V2)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs1, outs2 = [], []
    for _ in range(3):
        with torch.cuda.stream(s1):
            outs1.append(c1.saliency_maps(V1))
        with torch.cuda.stream(s2):
            outs2.append(c2.saliency_maps(V2))
    torch.cuda.synchronize()
    for got in outs1:
        for a, b in zip(got, ref1):
            assert torch.equal(a, b)
    for got in outs2:
        for a, b in zip(got, ref2):
            assert torch.equal(a, b)

"""The fused path inside a HIP graph: sal_saliency with a caller workspace allocates and
synchronises nothing, so it can be captured once and replayed.  Every replay (with eager
work and synchronisations between replays, and new data copied into the captured input)
must equal the eager call bit for bit."""
import pytest
import torch

from paper_1901_11095_amd import sal, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("L,prec,stride", [(8, sal.FP32, 1), (16, sal.BF16_SPLIT, 1), (5, sal.FP32, 1),
                                           (8, sal.FP32, 2)])
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

"""The batched build + queries captured in a HIP graph: every replay gives
the eager result, with eager library work and synchronisations between
replays."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def test_batch_graph_replays_match_eager():
    import torch
    import paper_2103_15217_amd as et
    dev = torch.device("cuda", 0)
    b = gen.forest_batch(300, seed=4, log2_min=3, log2_max=13, qlog2_min=2, qlog2_max=9)
    d = lambda a, t=torch.int32: torch.from_numpy(np.ascontiguousarray(a)).to(dev, t)
    parent, offs = d(b["parent"]), d(b["offsets"], torch.int64)
    qt, qx, qy = d(b["qtree"]), d(b["qx"]), d(b["qy"])
    ctx = et.Context()
    eager = et.et_tree_build_batch(parent, offs, ctx=ctx)
    want = eager.lca_batch(qt, qx, qy).cpu().numpy()
    eager.free()
    g = et.BatchGraph(parent, offs, qt, qx, qy, ctx=ctx)
    other_ctx = et.Context()
    for rep in range(4):
        g.out.fill_(-7)
        got = g.replay().cpu().numpy()
        assert np.array_equal(got, want), rep
        # unrelated eager work between replays (its own context)
        t = et.et_tree_build(d(gen.random_tree(5000, 3, seed=rep)), ctx=other_ctx)
        t.lca(qx[:100] % 5000, qy[:100] % 5000)
        t.free()
        torch.cuda.synchronize()
    ctx.check()
    other_ctx.check()
    g.close()


def test_bridges_batch_graph_replays_match_eager():
    import torch
    import paper_2103_15217_amd as et
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(9)
    graphs = []
    for t in range(120):
        n = int(2 ** rng.uniform(2, 11))
        graphs.append(gen.random_multigraph(n, int(n * rng.uniform(0.5, 3)), seed=t))
    d = lambda a, t=torch.int32: torch.from_numpy(np.ascontiguousarray(a)).to(dev, t)
    rows = d(np.concatenate([g[0] for g in graphs]))
    cols = d(np.concatenate([g[1] for g in graphs]))
    slots = [len(g[1]) for g in graphs]
    voff = d(np.concatenate([[0], np.cumsum([len(g[0]) - 1 for g in graphs])]), torch.int64)
    soff = d(np.concatenate([[0], np.cumsum(slots)]), torch.int64)
    ctx = et.Context()
    want_mask, spans, want_counts = et.et_bridges_batch(row_ptr=rows, col=cols, voff=voff, soff=soff, slots=slots,
                                                        ctx=ctx)
    want_mask, want_counts = want_mask.cpu().numpy(), want_counts.cpu().numpy()
    ctx.check()
    ctx.close()
    g = et.BridgesBatchGraph(rows, cols, voff, soff, slots)
    assert g.spans == spans
    other_ctx = et.Context()
    for rep in range(4):
        g.mask.fill_(-7)
        g.counts.fill_(-7)
        mask, counts = g.replay()
        assert np.array_equal(mask.cpu().numpy(), want_mask), rep
        assert np.array_equal(counts.cpu().numpy(), want_counts), rep
        # unrelated eager work between replays (its own context)
        rp, col = gen.random_multigraph(3000, 6000, seed=rep)
        et.et_bridges(d(rp), d(col), ctx=other_ctx)
        torch.cuda.synchronize()
    g.ctx.check()
    other_ctx.check()
    g.close()

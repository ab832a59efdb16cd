"""Serving loop: every job's result is the same alone (plain executor) and in
the mix (continuous batching with resident trees, batched builds and
overlapping streams), and LCA results match the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(oracle_mod):
    import torch
    from paper_2103_15217_amd import serve
    dev = torch.device("cuda", 0)
    pool = serve.make_pool(seed=3, trees=12, graphs=4, tree_log2=(4, 15), graph_log2=(8, 13))
    dpool = serve.upload_pool(pool, dev)
    jobs = serve.make_trace(pool, rate=20000, duration=0.03, seed=3, qlog2=(0, 9))
    assert len(jobs) > 200
    serve.upload_trace(jobs, dev)
    plain = serve.PlainExecutor(dpool, keep_results=True)
    plain.run(jobs)
    # a small memory budget forces evictions and re-builds in the mix
    served = serve.ServedExecutor(dpool, streams=3, budget_bytes=1 << 24, keep_results=True, max_batch=5)
    stats = served.run(jobs)
    served.close()
    assert stats["jobs"] == len(jobs)
    for j in jobs:
        a, b = plain.results[j.jid].numpy(), served.results[j.jid].numpy()
        assert np.array_equal(a, b), (j.jid, j.kind)
    for j in [j for j in jobs if j.kind == "lca"][:20]:
        want = oracle_mod.lca_offline(pool["trees"][j.item], j.qx.cpu().numpy(), j.qy.cpu().numpy())
        assert np.array_equal(served.results[j.jid].numpy(), want)
    for j in [j for j in jobs if j.kind == "bridges"][:5]:
        rp, col = pool["graphs"][j.item]
        ref, _ = oracle_mod.bridges(rp, col)
        assert np.array_equal(served.results[j.jid].numpy().view(np.uint32)[: len(ref)], ref)

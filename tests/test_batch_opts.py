"""Host side of the batch binding: per-problem options (one value for all
problems or one per problem) and the PlasmaTree domain-size cap, and the
batch autotuner's tile-size rules."""

import paper_1104_4475_amd as tqr
from paper_1104_4475_amd.api import _batch_opts, batch_nb_rules


def test_batch_options_per_problem_and_capped_domains():
    shapes, nbs = [(256, 32), (4096, 64), (1024, 128)], [32, 64, 64]
    o = _batch_opts(shapes, nbs, tqr.TREE_PLASMA, 16, tqr.KERN_TS, 1)
    assert [x.bs for x in o] == [8, 16, 16]  # 256 / 32 = 8 tile rows
    assert all(x.tree == tqr.TREE_PLASMA and x.kernels == tqr.KERN_TS and x.upd == 1 for x in o)
    assert [(x.m, x.n, x.nb) for x in o] == [(256, 32, 32), (4096, 64, 64), (1024, 128, 64)]
    o = _batch_opts(shapes, nbs, [tqr.TREE_GREEDY, tqr.TREE_PLASMA, tqr.TREE_FLAT], [1, 32, 1],
                    [tqr.KERN_TT, tqr.KERN_TS, tqr.KERN_TS], 0)
    assert [x.tree for x in o] == [tqr.TREE_GREEDY, tqr.TREE_PLASMA, tqr.TREE_FLAT]
    assert [x.bs for x in o] == [1, 32, 1]  # Greedy's bs is not a domain size: left as given
    assert [x.kernels for x in o] == [tqr.KERN_TT, tqr.KERN_TS, tqr.KERN_TS]


def test_batch_tile_size_rules():
    r = batch_nb_rules([(512, 64), (256, 32), (1024, 128), (192, 64)])
    assert r["nb 64 where it divides"] == [64, 32, 64, 64]
    assert r["nb 32"] == [32, 32, 32, 32]

"""GPU parity of the Boruvka minimum spanning forest (the Atomic construct's
workload) against the CPU oracle (Kruskal under the same total edge order,
pinned by brute force and scipy): the forest weight, the per-entry forest
marks and the per-vertex tree labels must match bit for bit, with every
compilation of the atomic section (packed 64-bit atomicMin, blocking CAS
lock, ticket lock), several block sizes, disconnected graphs, ties, hubs,
long paths and a relabelled upload."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_05707_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def irgl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1607_05707_amd import irgl as mod
    return mod


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _path(n):
    src = list(range(n - 1)) + list(range(1, n))
    dst = list(range(1, n)) + list(range(n - 1))
    w = [1 + (i * 7) % 13 for i in range(n - 1)] * 2
    return gg.from_edges(n, src, dst, w, name=f"path{n}")


def _check(irgl, g, hg, cfg):
    _say(f"mst {g.name} cfg={cfg}")
    weight, comp, in_forest, st = irgl.mst(hg, cfg=cfg)
    ref_w, ref_f, ref_c, ref_ne = oracle.kruskal(*g.numpy())
    assert weight == ref_w, (g.name, cfg)
    np.testing.assert_array_equal(in_forest.cpu().numpy(), ref_f, err_msg=f"{g.name} {cfg}")
    np.testing.assert_array_equal(comp.cpu().numpy(), ref_c, err_msg=f"{g.name} {cfg}")
    assert st["frontier_edges"] == ref_ne
    assert st["status"] == 0
    return st


def _dev(g):
    return g.to(torch.device("cuda:0"))


GRAPHS = [
    lambda: gg.rmat(12, seed=81, weight_seed=82, wmax=255),
    lambda: gg.config_road(width=64),
    lambda: gg.uniform_random(3000, 8.0, seed=83, weight_seed=84, wmax=1000),
    lambda: gg.uniform_random(2500, 0.8, seed=85, weight_seed=86, wmax=3),   # forest, many ties
    lambda: gg.grid2d(40, 30, weight_seed=87, wmax=1),                        # all weights equal
    lambda: _path(700),
]


@pytest.mark.parametrize("lock", [0, 1, 2])
def test_mst_matches_oracle(irgl, lock):
    for make in GRAPHS:
        g = _dev(make())
        hg = irgl.upload(g)
        for cfg in ({"lock": lock}, {"lock": lock, "block": 1024}, {"lock": lock, "block": 512, "barrier": 1}):
            _check(irgl, g, hg, cfg)


def test_mst_hubs_relabelled_and_larger(irgl):
    g = _dev(gg.rmat(16, seed=88, weight_seed=89, wmax=255))
    st = _check(irgl, g, irgl.upload(g), None)
    assert st["iterations"] >= 2
    # a relabelled handle: the results still refer to the caller's ids and entries
    _check(irgl, g, irgl.upload(g, reorder=True), {"lock": 1})
    # a hub (star) contended by every vertex in round 0, with equal weights
    n = 5000
    star = _dev(gg.from_edges(n, [0] * (n - 1) + list(range(1, n)), list(range(1, n)) + [0] * (n - 1),
                              [5] * (2 * (n - 1)), name="star"))
    for lock in (0, 1, 2):
        _check(irgl, star, irgl.upload(star), {"lock": lock})


def test_mst_edge_cases_and_errors(irgl):
    one = _dev(gg.from_edges(1, [], [], [], name="single"))
    w, comp, f, st = irgl.mst(irgl.upload(one))
    assert w == 0 and comp.cpu().tolist() == [0]
    iso = _dev(gg.from_edges(6, [1, 2], [2, 1], [9, 9], name="isolated"))
    _check(irgl, iso, irgl.upload(iso), {"lock": 2})
    unweighted = _dev(gg.grid2d(8, 8))
    hu = irgl.upload(unweighted)
    with pytest.raises(irgl.IrglError) as e:
        irgl.mst(hu)
    assert e.value.status == irgl.IRGL_ERR_NO_WEIGHTS
    g = _dev(gg.rmat(10, seed=90, weight_seed=91))
    hg = irgl.upload(g)
    with pytest.raises(irgl.IrglError) as e:
        irgl.mst(hg, cfg={"lock": 7})
    assert e.value.status == irgl.IRGL_ERR_CONFIG
    weight = torch.zeros(1, dtype=torch.int64, device=g.row_ptr.device)
    small = torch.empty(irgl.irgl_mst_workspace_bytes(hg) - 1, dtype=torch.uint8, device=g.row_ptr.device)
    with pytest.raises(irgl.IrglError) as e:
        irgl.irgl_mst(hg, weight, ws=small)
    assert e.value.status == irgl.IRGL_ERR_WORKSPACE_TOO_SMALL
    # an edge without its reverse is reported from the device
    d = _dev(gg.from_edges(4, [0, 1, 2, 2], [1, 0, 3, 0], [1, 1, 2, 5], name="asymmetric"))
    with pytest.raises(irgl.IrglError) as e:
        irgl.mst(irgl.upload(d, flags=0))
    assert e.value.status == irgl.IRGL_ERR_INVALID_GRAPH

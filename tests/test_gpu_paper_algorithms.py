"""GPU parity of the paper's Algorithms 1-4 (plan option `algorithm`) against
the FP64 oracle: the per-joint walk, barrier-synchronous pointer jumping,
64-joint blocks with the walk over out-of-block partials, and the window of
8 with hops of 8.  Same tolerances as the library's own scan."""
import numpy as np
import pytest
import torch

from paper_2505_06703_amd import hs
from paper_2505_06703_amd import workloads as wl

from parity import check_global, check_skin, inverse_binds, reference

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ALGS = [hs.HS_ALG_WALK, hs.HS_ALG_JUMP, hs.HS_ALG_BLOCKS, hs.HS_ALG_COMPRESSED]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _mixed():
    """Chains of 1..1024 joints, a star, a forest and an empty character."""
    rng = np.random.default_rng(9)
    parts = [np.arange(-1, n - 1, dtype=np.int32) for n in (1, 63, 64, 65, 200, 1024)]
    star = np.zeros(700, np.int32)
    star[0] = -1
    parts += [star, np.zeros(0, np.int32), np.array([-1, 0, -1, 2, 2, -1], np.int32)]
    par = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    q, t, s = wl.random_pose(rng, par.size, max_angle=0.1)
    # mildly non-uniform scale: products along the 1024-joint chain stay of
    # order one (wider ranges compound to 1e9 and leave fp32's range of
    # absolute tolerances)
    s = rng.uniform(0.97, 1.03, s.shape).astype(np.float32)
    return wl.Batch("mixed", off, par, q, t, s, q, t, s)


@pytest.mark.parametrize("alg", ALGS)
@pytest.mark.parametrize("name", ["depth15", "depth120", "plain", "deep", "hetero", "mixed"])
def test_paper_algorithm_matches_oracle(alg, name):
    b = {"depth15": lambda: wl.depth_sweep(num_characters=24, depth=15, templates=8),
         "depth120": lambda: wl.depth_sweep(num_characters=24, depth=120, templates=8),
         "plain": lambda: wl.plain_scan(num_characters=16),
         "deep": lambda: wl.deep_forward(num_characters=6),
         "hetero": lambda: wl.heterogeneous(num_characters=60, hi=1500, chain_fraction=0.05),
         "mixed": _mixed}[name]()
    plan = hs.Plan(b.offsets, b.parents, algorithm=alg)
    info = plan.info
    assert info["tile_joints"] <= 1024 and info["waves_per_tile"] == 16
    G, _ = hs.hs_scan_forward(plan, dev(b.quat), dev(b.trans), dev(b.scale))
    torch.cuda.synchronize()
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, f"algorithm {alg} on {name}")


@pytest.mark.parametrize("alg", ALGS)
def test_paper_algorithm_fused_skin_and_graph(alg):
    b = wl.plain_scan(num_characters=8)
    inv = inverse_binds(b)
    plan = hs.Plan(b.offsets, b.parents, algorithm=alg)
    q, t, s = dev(b.quat), dev(b.trans), dev(b.scale)
    G = torch.empty((b.num_joints, 4, 4), device=DEV)
    S = torch.empty_like(G)
    g = hs.ForwardGraph(plan, q, t, s, global_out=G, inv_bind=dev(inv), skin_out=S)
    g.launch()
    torch.cuda.synchronize()
    Gr, lam, _ = reference(b)
    check_global(G.cpu().numpy(), Gr, lam, f"algorithm {alg} graph")
    check_skin(S.cpu().numpy(), Gr, inv, lam, f"algorithm {alg} skin")


def test_paper_algorithm_options_are_validated():
    b = wl.plain_scan(num_characters=2)
    with pytest.raises(hs.HSError):
        hs.Plan(b.offsets, b.parents, algorithm=7)
    with pytest.raises(hs.HSError):
        hs.Plan(b.offsets, b.parents, algorithm=hs.HS_ALG_JUMP, chain_units=True)
    chain = np.arange(-1, 2999, dtype=np.int32)
    with pytest.raises(hs.HSError):
        hs.Plan(np.array([0, 3000], np.int64), chain, algorithm=hs.HS_ALG_WALK, strategy=hs.HS_STRATEGY_TILE)

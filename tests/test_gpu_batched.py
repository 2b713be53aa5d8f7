"""GPU tests of the batched uneven-tile pass (nk_myrtle_nngp_batched): every
tile bitwise equal to the one-block entry point on the same tile, sampled
entries of every tile against the FP64 oracle (normalised error <= 2e-5),
shared image arrays with different prefixes, symmetric tiles, padded
leading dimensions, the tuned schedule, and hipGraph capture with replays
checked one by one against the eager pass."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 2e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _tiles_from_shapes(pool_a, pool_b, shapes, sym_every=0, pad=0):
    """Tiles over prefixes of two image pools: (x1 tensor view, x2 or None, out)."""
    tiles = []
    for t, (n1, n2) in enumerate(shapes):
        if sym_every and t % sym_every == 0:
            x1 = pool_a[:n1]
            out = torch.full((n1, n1 + pad), float("nan"), device="cuda")
            tiles.append((x1, None, out))
        else:
            out = torch.full((n1, n2 + pad), float("nan"), device="cuda")
            tiles.append((pool_a[:n1], pool_b[:n2], out))
    return tiles


def _oracle_sample(xa, xb, tiles, depth, rng, per_tile):
    """Oracle values at seeded entries of every tile: list of (tile, rows, cols, values, d1, d2)."""
    net = oracle.Myrtle(depth)
    qa, da = oracle.myrtle_self(xa, net)
    qb, db = oracle.myrtle_self(xb, net)
    res = []
    for t, (x1, x2, out) in enumerate(tiles):
        n1 = x1.shape[0]
        n2 = n1 if x2 is None else x2.shape[0]
        r = rng.integers(0, n1, per_tile)
        c = rng.integers(0, n2, per_tile)
        if x2 is None:
            v = oracle.myrtle_pairs(xa, xa, np.stack([r, c], 1), net, qa, qa)
            res.append((t, r, c, v, da[r], da[c]))
        else:
            v = oracle.myrtle_pairs(xa, xb, np.stack([r, c], 1), net, qa, qb)
            res.append((t, r, c, v, da[r], db[c]))
    return res


def test_batched_small_uneven_tiles_match_plain_and_oracle(nk):
    depth = (2, 1, 1)
    xa_n = synth.iid_images(80, 8, 8, 3, 11)
    xb_n = synth.iid_images(70, 8, 8, 3, 12)
    xa, xb = _gpu(xa_n), _gpu(xb_n)
    shapes = [(17, 40), (1, 1), (64, 3), (80, 70), (33, 33), (5, 69), (40, 17), (80, 1)]
    tiles = _tiles_from_shapes(xa, xb, shapes, sym_every=3, pad=5)
    _say(f"batched 8x8 Myrtle-5: {len(tiles)} tiles")
    nk.myrtle_nngp_batched(tiles, depth)
    torch.cuda.synchronize()
    for t, (x1, x2, out) in enumerate(tiles):
        n2 = x1.shape[0] if x2 is None else x2.shape[0]
        ref = nk.myrtle_nngp(x1, x2, depth).cpu().numpy()
        got = out[:, :n2].cpu().numpy()
        assert np.array_equal(got, ref), f"tile {t} differs from the one-block entry point"
        assert torch.isnan(out[:, n2:]).all(), f"tile {t} wrote past n2"
    rng = np.random.default_rng(13)
    for t, r, c, v, d1, d2 in _oracle_sample(xa_n, xb_n, tiles, depth, rng, 6):
        got = tiles[t][2].cpu().numpy()[r, c]
        err = float(np.max(np.abs(got - v) / np.sqrt(d1 * d2)))
        assert err <= TOL, f"tile {t}: {err:.2e}"
    cands, chosen = nk.batched_tuning(8, 3, depth)
    _say(f"  tuned: {chosen} of {len(cands)} candidates")
    sched = [c for c in cands if c["kind"] == "schedule"]
    shape = [c for c in cands if c["kind"] == "shape"]
    assert len(sched) >= 2
    assert any(c["chunk"] == chosen["chunk"] and c["pair_tile"] == chosen["pair_tile"]
               and c["persistent"] == chosen["persistent"] for c in sched)
    # kernel shape (pairs per workgroup of the 8x8 .. 2x2 stages) timed under
    # the chosen schedule; the faster one is kept
    assert sorted(c["wg_pairs_mult"] for c in shape) == [1, 2]
    assert all(c["chunk"] == chosen["chunk"] and c["pair_tile"] == chosen["pair_tile"]
               and c["persistent"] == chosen["persistent"] for c in shape)
    assert chosen["wg_pairs_mult"] == min(shape, key=lambda c: c["us_per_pair"])["wg_pairs_mult"]


@pytest.mark.parametrize("mult", [2, 1])
def test_batched_kernel_shapes_are_bitwise_equal(nk, mult):
    """Both kernel shapes of the stages of tiles of at most 16 x 16 (one or
    two pairs-per-workgroup multiples), fixed through
    nk_myrtle_batched_set_schedule, give the one-block entry point's values
    bit for bit, on uneven tiles with symmetric ones among them."""
    depth = (1, 2, 2)  # a network no other test tunes
    xa = _gpu(synth.correlated_images(40, 16, 16, 3, 2.0, 31))
    xb = _gpu(synth.correlated_images(33, 16, 16, 3, 2.0, 32))
    tiles = _tiles_from_shapes(xa, xb, [(40, 33), (9, 31), (25, 25), (40, 1), (3, 3), (17, 2)], sym_every=2, pad=3)
    nk.batched_set_schedule(16, 3, depth, chunk=512, pair_tile=8, persistent=1, wg_pairs_mult=mult)
    _say(f"batched 16x16 Myrtle-7, pairs-per-workgroup multiple {mult}")
    nk.myrtle_nngp_batched(tiles, depth)
    torch.cuda.synchronize()
    for t, (x1, x2, out) in enumerate(tiles):
        n2 = x1.shape[0] if x2 is None else x2.shape[0]
        ref = nk.myrtle_nngp(x1, x2, depth).cpu().numpy()
        got = out[:, :n2].cpu().numpy()
        assert np.array_equal(got, ref), f"tile {t} differs from the one-block entry point"
        assert torch.isnan(out[:, n2:]).all(), f"tile {t} wrote past n2"
    cands, chosen = nk.batched_tuning(16, 3, depth)
    assert cands == [] and chosen["wg_pairs_mult"] == mult


@pytest.mark.parametrize("persistent", [1, 0])
def test_batched_32x32_persistent_units_bitwise(nk, persistent):
    """The 32x32 stage with several pairs per workgroup in a row (persistent
    grid, 2048-pair chunks over 256 workgroups: about 8 pairs each; the
    pooling exchange's flags count on from pair to pair) and with one pair
    per workgroup, against the one-block entry point bit for bit."""
    depth = (2, 1, 1)  # a network no other test tunes at 32x32
    xa = _gpu(synth.correlated_images(48, 32, 32, 3, 3.0, 41))
    xb = _gpu(synth.correlated_images(44, 32, 32, 3, 3.0, 42))
    tiles = _tiles_from_shapes(xa, xb, [(48, 44), (9, 31), (30, 30), (48, 1), (3, 3), (17, 40)], sym_every=2, pad=2)
    nk.batched_set_schedule(32, 3, depth, chunk=2048, pair_tile=8, persistent=persistent, wg_pairs_mult=1)
    _say(f"batched 32x32 Myrtle-5 stage shapes, persistent {persistent}")
    nk.myrtle_nngp_batched(tiles, depth)
    torch.cuda.synchronize()
    for t, (x1, x2, out) in enumerate(tiles):
        n2 = x1.shape[0] if x2 is None else x2.shape[0]
        ref = nk.myrtle_nngp(x1, x2, depth).cpu().numpy()
        got = out[:, :n2].cpu().numpy()
        assert np.array_equal(got, ref), f"tile {t} differs from the one-block entry point"
        assert torch.isnan(out[:, n2:]).all(), f"tile {t} wrote past n2"


def test_batched_graph_replays_match_eager(nk):
    depth = (2, 2, 2)
    xa = _gpu(synth.correlated_images(48, 16, 16, 3, 2.0, 21))
    xb = _gpu(synth.correlated_images(40, 16, 16, 3, 2.0, 22))
    tiles = _tiles_from_shapes(xa, xb, [(48, 40), (7, 39), (30, 30), (48, 1), (12, 12)], sym_every=2)
    _say("batched 16x16 Myrtle-7 eager")
    nk.myrtle_nngp_batched(tiles, depth, graph=False)
    torch.cuda.synchronize()
    eager = [o.clone() for _, _, o in tiles]
    for rep in range(3):
        for _, _, o in tiles:
            o.fill_(float("nan"))
        _say(f"  graph pass {rep}")
        nk.myrtle_nngp_batched(tiles, depth, graph=True)
        torch.cuda.synchronize()
        # eager work on the same stream between replays
        junk = nk.myrtle_nngp(xa[:9], xb[:4], depth)
        torch.cuda.synchronize()
        del junk
        for t, (_, _, o) in enumerate(tiles):
            assert torch.equal(o, eager[t]), f"replay {rep}, tile {t} differs from the eager pass"


def test_batched_uneven_myrtle7_32x32_sample(nk):
    """The uneven-tile workload at reduced tile sides (U{32..256} instead of
    U{32..2048}; same generator, pools and network), >= 4 oracle entries per
    tile and bitwise agreement with the one-block entry point."""
    w = synth.WORKLOADS["myrtle7_uneven64"]
    depth = w["depth"]
    n_tiles = 16
    shapes = synth.uneven_tile_shapes(n_tiles, 32, 256, w["seeds"][2])
    pa = synth.correlated_images(256, 32, 32, 3, w["length"], w["seeds"][0])
    pb = synth.correlated_images(256, 32, 32, 3, w["length"], w["seeds"][1])
    xa, xb = _gpu(pa), _gpu(pb)
    tiles = _tiles_from_shapes(xa, xb, [tuple(int(v) for v in s) for s in shapes])
    _say(f"batched 32x32 Myrtle-7: {n_tiles} tiles, {sum(int(a) * int(b) for a, b in shapes)} pairs")
    nk.myrtle_nngp_batched(tiles, depth)
    torch.cuda.synchronize()
    for t in (0, 5, 11):
        x1, x2, out = tiles[t]
        ref = nk.myrtle_nngp(x1, x2, depth).cpu().numpy()
        assert np.array_equal(out.cpu().numpy(), ref)
    rng = np.random.default_rng(w["seeds"][2] + 1)
    for t, r, c, v, d1, d2 in _oracle_sample(pa, pb, tiles, depth, rng, 4):
        got = tiles[t][2].cpu().numpy()[r, c]
        err = float(np.max(np.abs(got - v) / np.sqrt(d1 * d2)))
        assert err <= TOL, f"tile {t}: {err:.2e}"


@pytest.mark.timeout(600)
def test_batched_full_uneven_tile_list_sampled(nk):
    """The uneven-tile workload at its stated size: 64 Myrtle-7 tiles with
    sides U{32..2048} over prefixes of two pools of 2048 32x32x3 images, one
    batched pass (hipGraph); 4 seeded oracle entries per tile, and the two
    smallest tiles bitwise equal to the one-block entry point."""
    w = synth.WORKLOADS["myrtle7_uneven64"]
    depth = w["depth"]
    shapes = [tuple(int(v) for v in s) for s in synth.uneven_tile_shapes(w["n_tiles"], w["lo"], w["hi"],
                                                                         w["seeds"][2])]
    pa = synth.correlated_images(w["pool"], 32, 32, 3, w["length"], w["seeds"][0])
    pb = synth.correlated_images(w["pool"], 32, 32, 3, w["length"], w["seeds"][1])
    xa, xb = _gpu(pa), _gpu(pb)
    tiles = _tiles_from_shapes(xa, xb, shapes)
    _say(f"batched full workload: {len(tiles)} tiles, {sum(a * b for a, b in shapes)} pairs")
    nk.myrtle_nngp_batched(tiles, depth, graph=True)
    torch.cuda.synchronize()
    _say("  batched pass done")
    small = sorted(range(len(shapes)), key=lambda t: shapes[t][0] * shapes[t][1])[:2]
    for t in small:
        x1, x2, out = tiles[t]
        assert np.array_equal(out.cpu().numpy(), nk.myrtle_nngp(x1, x2, depth).cpu().numpy()), f"tile {t}"
    rng = np.random.default_rng(w["seeds"][2] + 2)
    rows = [rng.integers(0, a, 4) for a, _ in shapes]
    cols = [rng.integers(0, b, 4) for _, b in shapes]
    ia = np.unique(np.concatenate(rows))
    ib = np.unique(np.concatenate(cols))
    net = oracle.Myrtle(depth)
    _say(f"  oracle: {len(ia) + len(ib)} self recursions, {4 * len(shapes)} entries")
    qa, da = oracle.myrtle_self(pa[ia], net)
    qb, db = oracle.myrtle_self(pb[ib], net)
    pos_a = {int(v): i for i, v in enumerate(ia)}
    pos_b = {int(v): i for i, v in enumerate(ib)}
    loc = np.array([[pos_a[int(r)], pos_b[int(c)]] for rr, cc in zip(rows, cols) for r, c in zip(rr, cc)])
    ref = oracle.myrtle_pairs(pa[ia], pb[ib], loc, net, qa, qb)
    got = np.concatenate([tiles[t][2][torch.as_tensor(rows[t]).cuda(), torch.as_tensor(cols[t]).cuda()].cpu().numpy()
                          for t in range(len(shapes))])
    err = float(np.max(np.abs(got - ref) / np.sqrt(da[loc[:, 0]] * db[loc[:, 1]])))
    _say(f"  normalised error over {len(ref)} entries: {err:.3e}")
    assert err <= TOL

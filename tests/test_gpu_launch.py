"""The fused launch: every length bucket in one kernel launch, tile shapes
(forced or autotuned) and replayed HIP graphs of whole sampling blocks.

Tile shapes only change which tiles share a workgroup and whether the
transform tables stay in LDS; each tile runs the same instructions on the
same data, so every shape must give bit-identical states.  A replayed graph
runs the same kernels as the eager path, so it too must be bit-identical,
replay after replay.
"""
import numpy as np
import pytest
import torch

from paper_1411_3487_amd import Context, inputs

pytestmark = pytest.mark.gpu

NU, TS = 0.35, 0.034
B_FAC = 1.0 / (1.0 - 2.0 * NU)
LENS = [64, 96, 128, 192, 256, 384, 512]
DTAU = {64: 10.0, 96: 10.0, 128: 50.0, 192: 50.0, 256: 100.0, 384: 100.0, 512: 100.0}


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def uneven(n, seed=2):
    beads = inputs.mixed_lengths(n, LENS, seed=seed)
    return beads, inputs.mixed_chains(beads, B_FAC, seed=seed)


def run_modes(chains, prec, n_steps, **kw):
    with Context(chains, seed=2, precision=prec) as ctx:
        ctx.set_params(LENS, [DTAU[m] for m in LENS], T_star=TS, nu=NU, **kw)
        ctx.step_modes(n_steps)
        return ctx.modes(), ctx.tiling()


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_all_lengths_share_one_launch_and_shapes_agree(prec):
    beads, chains = uneven(230)  # several tiles per length, ragged last tiles
    ref, til = run_modes(chains, prec, 6)
    print(prec, [(int(t["M"]), int(t["RT"]), int(t["JC"]), int(t["resident"]), int(t["tpw"]))
                 for t in til])
    assert [int(t["M"]) for t in til] == LENS
    for mode, tpw in [("resident", 1), ("resident", 2), ("resident", 3), ("streamed", 0)]:
        got, til2 = run_modes(chains, prec, 6, table_mode=mode, tiles_per_wg=tpw)
        for t in til2:
            if mode == "streamed" and t["RT"] >= 8:
                assert t["resident"] == 0 and t["tpw"] == 4
            if mode == "resident" and t["RT"] < 8:
                assert t["resident"] == 1 and t["tpw"] == tpw
        assert same(ref, got), (mode, tpw)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_autotuned_shapes_give_identical_states(prec):
    beads, chains = uneven(300)
    ref, _ = run_modes(chains, prec, 5)
    with Context(chains, seed=2, precision=prec) as ctx:
        ctx.set_params(LENS, [DTAU[m] for m in LENS], T_star=TS, nu=NU, autotune=True)
        rep = ctx.tuning_report()
        til = ctx.tiling()
        ctx.step_modes(5)
        got = ctx.modes()
    print(rep)
    assert rep.count("chosen") == len(LENS)
    assert all(t["item_us"] > 0 for t in til)
    assert same(ref, got)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_graph_replays_match_eager(prec):
    """Sampling every 10 steps; calls that start off a block boundary and end
    mid-block mix eager launches with replays.  After every call the state
    and the accumulators of the graph context equal the eager context's."""
    beads, chains = uneven(60)
    ctxs = []
    for graphs in (False, True):
        c = Context(chains, seed=2, precision=prec)
        c.set_params(LENS, [DTAU[m] for m in LENS], T_star=TS, nu=NU, sample_every=10,
                     use_graphs=graphs, corr_lags=4)
        ctxs.append(c)
    try:
        total = 0
        for n in (7, 23, 40, 30, 5, 25):
            for c in ctxs:
                c.step_modes(n)
            total += n
            torch.cuda.synchronize()
            eager, graph = [c.modes() for c in ctxs]
            assert same(eager, graph), n
            ae, ag = [c.accumulators() for c in ctxs]
            for x, y in zip(ae, ag):
                assert x["n_samples"] == y["n_samples"] == total // 10
                for k in ("bond", "L2", "msd_cm"):
                    assert x[k] == y[k], (n, k)
                assert np.array_equal(x["modes"], y["modes"])
                assert np.array_equal(x["corr"], y["corr"])
            assert ctxs[0].step == ctxs[1].step
    finally:
        for c in ctxs:
            c.close()


def test_graph_replays_single_length_benchmark_shape():
    """4096 x 256 bp, split BF16, observables every 100 steps."""
    B, M = 4096, 256
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    out = []
    for graphs in (False, True):
        with Context(pos, seed=1, precision="bf16x3") as c:
            c.set_params([M], [100.0], T_star=TS, nu=NU, sample_every=100, use_graphs=graphs)
            c.step_modes(300)
            out.append((c.modes(), c.accumulators()[0]))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1]["L2"] == out[1][1]["L2"] and out[0][1]["n_samples"] == 3


# Split tiles: one tile of 5 chains per workgroup, its bond rows and mode
# tiles divided among 4 (or, split-BF16 at RT = 8 and 16, 8) wavefronts that
# exchange amplitudes, forces and one normal per tile through LDS.  Each
# accumulator sees the same products in the same order as with one wavefront
# per tile, so the states agree bit for bit.  Lengths with RT = 4 (96, 128
# beads), 8 (256), 12 (384), 16 (512).
SPLIT_LENS = [96, 128, 256, 384, 512]
SPLIT_DTAU = {96: 10.0, 128: 50.0, 256: 100.0, 384: 100.0, 512: 100.0}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("kw", [{}, {"gamma_dot": 3e-6}, {"nonlinear": False}],
                         ids=["nonlinear", "shear", "linear"])
def test_split_tiles_bit_identical_to_one_wavefront_per_tile(prec, kw):
    beads = inputs.mixed_lengths(61, SPLIT_LENS, seed=3)  # ragged last tiles
    chains = inputs.mixed_chains(beads, B_FAC, seed=3)
    runs = {}
    for mode in ("split", "resident", "streamed"):
        with Context(chains, seed=4, precision=prec) as ctx:
            ctx.set_params(SPLIT_LENS, [SPLIT_DTAU[m] for m in SPLIT_LENS], T_star=TS, nu=NU,
                           table_mode=mode, **kw)
            til = ctx.tiling()
            ctx.step_modes(7)
            runs[mode] = (ctx.modes(), til)
    print(prec, kw, [(int(t["M"]), int(t["RT"]), int(t["JC"]), int(t["split"]))
                     for t in runs["split"][1]])
    assert all(int(t["split"]) == 1 and int(t["items"]) == -(-int(t["n_chains"]) // 5)
               for t in runs["split"][1])
    assert all(int(t["split"]) == 0 for m in ("resident", "streamed") for t in runs[m][1])
    assert same(runs["split"][0], runs["resident"][0])
    assert same(runs["split"][0], runs["streamed"][0])


@pytest.mark.parametrize("kw", [{}, {"gamma_dot": 3e-6}, {"nonlinear": False}],
                         ids=["nonlinear", "shear", "linear"])
def test_split_tiles_of_8_wavefronts_bit_identical(kw):
    """table_mode = 4 (split-BF16): RT = 8 (256 beads) and RT = 16 (512) on
    tiles split over 8 wavefronts, in a kernel of their own launched after
    the one of the other lengths' tiles; states equal to 4-wavefront split
    tiles and to one wavefront per tile, with ragged last tiles."""
    beads = inputs.mixed_lengths(61, SPLIT_LENS, seed=3)
    chains = inputs.mixed_chains(beads, B_FAC, seed=3)
    runs = {}
    for mode in ("split8", "split", "streamed"):
        with Context(chains, seed=4, precision="bf16x3") as ctx:
            ctx.set_params(SPLIT_LENS, [SPLIT_DTAU[m] for m in SPLIT_LENS], T_star=TS, nu=NU,
                           table_mode=mode, **kw)
            til = ctx.tiling()
            ctx.step_modes(7)
            runs[mode] = (ctx.modes(), til)
    til8 = runs["split8"][1]
    print(kw, [(int(t["M"]), int(t["RT"]), int(t["split"])) for t in til8])
    assert [int(t["split"]) for t in til8] == [2 if int(t["RT"]) in (8, 16) else 0
                                               for t in til8]
    assert all(int(t["items"]) == -(-int(t["n_chains"]) // 5) for t in til8 if t["split"])
    assert same(runs["split8"][0], runs["split"][0])
    assert same(runs["split8"][0], runs["streamed"][0])


def test_split_tiles_of_8_wavefronts_mixed_plan_under_graphs():
    """A plan of both kernels (8-wavefront split tiles for 256 and 512
    beads, one-wavefront tiles for the other lengths) replayed as sampling
    blocks with deferred observables equals the eager default shapes:
    states, accumulators and correlators."""
    beads = inputs.mixed_lengths(61, SPLIT_LENS, seed=5)
    chains = inputs.mixed_chains(beads, B_FAC, seed=5)
    res = []
    for mode, graphs in (("split8", True), ("auto", False)):
        with Context(chains, seed=7, precision="bf16x3") as c:
            c.set_params(SPLIT_LENS, [SPLIT_DTAU[m] for m in SPLIT_LENS], T_star=TS, nu=NU,
                         sample_every=10, use_graphs=graphs, table_mode=mode, corr_lags=3)
            if mode == "split8":
                assert sorted({int(t["split"]) for t in c.tiling()}) == [0, 2]
            c.step_modes(45)
            c.step_modes(30)
            res.append((c.modes(), c.accumulators()))
    assert same(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert a["n_samples"] == b["n_samples"] == 7
        for k in ("bond", "L2", "msd_cm"):
            assert a[k] == b[k], k
        assert np.array_equal(a["modes"], b["modes"])
        assert np.array_equal(a["corr"], b["corr"])


def test_split_tiles_of_8_wavefronts_graphs_and_fp32():
    """8-wavefront split tiles under replayed sampling blocks equal the eager
    one-wavefront tiles (states, accumulators, correlators); in FP32 the form
    does not exist and table_mode = 4 leaves the default shape."""
    B, M = 300, 512
    pos = inputs.straight_chains(B, M, B_FAC, seed=6, random_orientation=True)
    res = []
    for mode, graphs in (("split8", True), ("streamed", False)):
        with Context(pos, seed=6, precision="bf16x3") as c:
            c.set_params([M], [100.0], T_star=TS, nu=NU, sample_every=10, use_graphs=graphs,
                         table_mode=mode, corr_lags=3)
            assert int(c.tiling()[0]["split"]) == (2 if mode == "split8" else 0)
            c.step_modes(45)
            c.step_modes(30)
            res.append((c.modes(), c.accumulators()[0]))
    assert same(res[0][0], res[1][0])
    a, b = res[0][1], res[1][1]
    assert a["n_samples"] == b["n_samples"] == 7
    for k in ("bond", "L2", "msd_cm"):
        assert a[k] == b[k], k
    assert np.array_equal(a["corr"], b["corr"])
    with Context(pos[:20], seed=6, precision="fp32") as c:
        c.set_params([M], [100.0], T_star=TS, nu=NU, table_mode="split8")
        assert int(c.tiling()[0]["split"]) == 0


@pytest.mark.parametrize("B,M,dtau", [(1024, 128, 50.0), (1024, 512, 100.0)])
def test_split_tiles_at_batched_sizes(B, M, dtau):
    """The 1024-chain configurations, where the automatic shape (fewer tiles
    than compute units) is the split tile."""
    pos = inputs.straight_chains(B, M, B_FAC, seed=1, random_orientation=True)
    out = []
    for mode in ("auto", "streamed" if M > 256 else "resident"):
        with Context(pos, seed=1, precision="bf16x3") as c:
            c.set_params([M], [dtau], T_star=TS, nu=NU, table_mode=mode)
            assert (int(c.tiling()[0]["split"]) >= 1) == (mode == "auto")
            c.step_modes(5)
            out.append(c.modes())
    assert same(out[0], out[1])


def test_split_tiles_graph_replays_and_observables():
    """Split tiles under replayed sampling blocks: states and accumulators
    equal to the eager run of the other shape."""
    B, M = 300, 256
    pos = inputs.straight_chains(B, M, B_FAC, seed=6, random_orientation=True)
    res = []
    for mode, graphs in (("split", True), ("resident", False)):
        with Context(pos, seed=6, precision="bf16x3") as c:
            c.set_params([M], [100.0], T_star=TS, nu=NU, sample_every=10, use_graphs=graphs,
                         table_mode=mode, corr_lags=3)
            c.step_modes(45)
            c.step_modes(30)
            res.append((c.modes(), c.accumulators()[0]))
    assert same(res[0][0], res[1][0])
    a, b = res[0][1], res[1][1]
    assert a["n_samples"] == b["n_samples"] == 7
    for k in ("bond", "L2", "msd_cm"):
        assert a[k] == b[k], k
    assert np.array_equal(a["modes"], b["modes"])
    assert np.array_equal(a["corr"], b["corr"])


def test_table_mode_split_where_it_exists_and_bad_modes_rejected():
    """table_mode = 3 puts the lengths with RT = 4, 8, 12, 16 on split tiles
    and leaves the others on their default shape; 5 is rejected."""
    from paper_1411_3487_amd import DMError
    beads, chains = uneven(40)
    with Context(chains, seed=2, precision="bf16x3") as ctx:
        with pytest.raises(DMError):
            ctx.set_params(LENS, [DTAU[m] for m in LENS], T_star=TS, nu=NU, table_mode=5)
        ctx.set_params(LENS, [DTAU[m] for m in LENS], T_star=TS, nu=NU, table_mode="split")
        til = ctx.tiling()
        assert [int(t["RT"]) for t in til] == [2, 4, 4, 6, 8, 12, 16]
        assert [int(t["split"]) for t in til] == [0, 1, 1, 0, 1, 1, 1]
        assert all(int(t["tpw"]) == 1 and int(t["resident"]) == 0 for t in til if t["split"])
        ctx.step_modes(3)
        assert np.all(np.isfinite(ctx.chain_observables()))


def test_fp64_graph_replays_match_eager_steps():
    """The FP64 plain form's sampling blocks replayed as a HIP graph (each
    update reading its Philox step from the device counter) give the same
    bits as eager steps, with eager work and synchronisations between the
    replays, for two length buckets."""
    beads = [64, 96, 64, 96, 96]
    chains = [inputs.straight_chains(1, m, B_FAC, seed=60 + i)[0] for i, m in enumerate(beads)]
    out = {}
    for graphs in (False, True):
        with Context(chains, seed=6, precision="fp64") as ctx:
            ctx.set_params([64, 96], [10.0, 10.0], T_star=TS, nu=NU, sample_every=25,
                           use_graphs=graphs)
            ctx.step_modes(100)          # 4 replayed blocks
            torch.cuda.synchronize()
            ctx.step_modes(7)            # eager, partial block
            ctx.step_modes(18)           # completes the block eagerly
            ctx.step_modes(75)           # 3 more replays
            out[graphs] = (ctx.modes(), ctx.accumulators())
    for c in range(len(beads)):
        assert np.array_equal(out[True][0][c], out[False][0][c]), c
    for a, b in zip(out[True][1], out[False][1]):
        assert a["n_samples"] == b["n_samples"] == 8
        for k in ("bond", "L2", "dmid2", "msd_cm"):
            assert a[k] == b[k], k
        assert np.array_equal(a["modes"], b["modes"])

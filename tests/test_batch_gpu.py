"""GPU parity of the batched persistent plan (HIP graph) and the autotuner."""

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_close, dequantized, normalized_errors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1611_02665_amd import binding as B  # noqa: E402

KIND_COMPS = {"v": ("v",), "vgl": ("v", "g", "l"), "vgh": ("v", "g", "h")}


def _outs(kind, npos, ldo, fill=12345.0):
    d = torch.device("cuda")
    o = {"v": torch.full((npos, ldo), fill, device=d)}
    if kind != "v":
        o["g"] = torch.full((npos, 3, ldo), fill, device=d)
    if kind == "vgl":
        o["l"] = torch.full((npos, ldo), fill, device=d)
    if kind == "vgh":
        o["h"] = torch.full((npos, 6, ldo), fill, device=d)
    return o


def _lh(kind, o):
    return o.get("l") if kind == "vgl" else o.get("h")


def _host(o, n):
    return {k: t.cpu().numpy()[..., :n].astype(np.float64) for k, t in o.items()}


class Tables:
    def __init__(self, shapes, dtype="f32", seed_stream=50):
        self.coefs, self.handles, self.boxes = [], [], []
        for i, s in enumerate(shapes):
            c = synth.coef_table(*s, stream=seed_stream + 2 * i)
            box = (1.0 + 0.1 * i, 1.0, 1.0 - 0.05 * i)
            self.coefs.append(c)
            self.boxes.append(box)
            self.handles.append(B.spline_table_create(*s, c, dtype, box))

    def close(self):
        for h in self.handles:
            B.spline_table_destroy(h)


SMALL = [(6, 6, 6, 64), (7, 5, 9, 200), (8, 8, 8, 300), (5, 5, 5, 1000)]
SMALL_NPOS = [7, 50, 130, 300]


@pytest.mark.parametrize("kind", ["v", "vgl", "vgh"])
@pytest.mark.parametrize("tile", [(2, 2, 1, 64, 0), (4, 1, 2, 256, 1), (1, 4, 1, 1000, 2),
                                  (2, 1, 2, 0, 3), (1, 2, 2, 0, 4), (2, 2, 1, 128, 4)])
def test_batch_plan_replays(kind, tile):
    T = Tables(SMALL)
    dev = torch.device("cuda")
    try:
        pos = [synth.positions(n, stream=60 + i) * 3 - 1 for i, n in enumerate(SMALL_NPOS)]
        pos = [p * np.array(T.boxes[i])[:, None] for i, p in enumerate(pos)]
        pd = [torch.from_numpy(p).to(dev) for p in pos]
        ldo = [s[3] + 3 for s in SMALL]
        outs = [_outs(kind, n, l) for n, l in zip(SMALL_NPOS, ldo)]
        plan = B.spline_batch_plan_create(
            T.handles, SMALL_NPOS, kind, pd, [o["v"] for o in outs],
            [o.get("g") for o in outs], [_lh(kind, o) for o in outs], ldo, tile=tile)
        assert B.spline_batch_plan_tile(plan).as_tuple()[:5] == tile
        refs = [oracle.evaluate(kind, T.coefs[i], pos[i], box=T.boxes[i]) for i in range(4)]
        for rep in range(3):
            for o in outs:  # eager work between replays
                for t in o.values():
                    t.fill_(float(rep))
            torch.cuda.synchronize()
            B.spline_batch_execute(plan)
            torch.cuda.synchronize()
            for i in range(4):
                n = SMALL[i][3]
                got = _host(outs[i], n)
                assert_close(kind, got, refs[i], label=f"replay {rep} table {i}")
                for t in outs[i].values():  # padding columns untouched by the plan
                    assert torch.all(t[..., n:] == float(rep))
        # rebind table 2 to new positions and outputs
        pos2 = synth.positions(SMALL_NPOS[2], stream=70) * np.array(T.boxes[2])[:, None]
        pd2 = torch.from_numpy(pos2).to(dev)
        o2 = _outs(kind, SMALL_NPOS[2], ldo[2])
        B.spline_batch_rebind(plan, 2, pd2, o2["v"], o2.get("g"), _lh(kind, o2))
        B.spline_batch_execute(plan)
        torch.cuda.synchronize()
        ref2 = oracle.evaluate(kind, T.coefs[2], pos2, box=T.boxes[2])
        assert_close(kind, _host(o2, SMALL[2][3]), ref2, label="rebound")
        B.spline_batch_plan_destroy(plan)
    finally:
        T.close()


def test_batch_plan_autotuned_and_wisdom(tmp_path):
    T = Tables(SMALL[:3])
    dev = torch.device("cuda")
    wisdom = str(tmp_path / "wisdom.txt")
    try:
        npos = SMALL_NPOS[:3]
        pos = [synth.positions(n, stream=80 + i) * np.array(T.boxes[i])[:, None]
               for i, n in enumerate(npos)]
        pd = [torch.from_numpy(p).to(dev) for p in pos]
        ldo = [s[3] for s in SMALL[:3]]
        outs = [_outs("vgh", n, l) for n, l in zip(npos, ldo)]
        args = (T.handles, npos, "vgh", pd, [o["v"] for o in outs], [o["g"] for o in outs],
                [o["h"] for o in outs], ldo)
        plan = B.spline_batch_plan_create(*args, tile=None, wisdom_path=wisdom)
        tile = B.spline_batch_plan_tile(plan)
        assert tile.grid >= 0 and tile.split in (0, 1)  # a full or a persistent grid
        text = open(wisdom).read()
        assert text.startswith("batch|") and "+" in text
        B.spline_batch_execute(plan)
        torch.cuda.synchronize()
        for i in range(3):
            ref = oracle.evaluate("vgh", T.coefs[i], pos[i], box=T.boxes[i])
            assert_close("vgh", _host(outs[i], SMALL[i][3]), ref, label=f"tuned table {i}")
        B.spline_batch_plan_destroy(plan)
        # a second plan with the same shapes takes the tile from the wisdom file
        plan2 = B.spline_batch_plan_create(*args, tile=None, wisdom_path=wisdom)
        assert B.spline_batch_plan_tile(plan2).as_tuple() == tile.as_tuple()
        assert open(wisdom).read() == text  # no new sweep appended
        B.spline_batch_plan_destroy(plan2)
    finally:
        T.close()


def test_batch_plan_rejects_mixed_dtypes():
    a = Tables([(4, 4, 4, 32)], "f32")
    b = Tables([(4, 4, 4, 32)], "f16", seed_stream=90)
    try:
        d = torch.device("cuda")
        p = torch.zeros(3, 4, dtype=torch.float64, device=d)
        v = torch.zeros(4, 32, device=d)
        with pytest.raises(B.BsplineError) as e:
            B.spline_batch_plan_create(a.handles + b.handles, [4, 4], "v", [p, p], [v, v],
                                       ldo=[32, 32], tile=(1, 1, 1, 8, 0))
        assert e.value.status == B.BSPL_EUNSUPPORTED
    finally:
        a.close()
        b.close()


def test_autotune_single_table(tmp_path):
    coef = synth.coef_table(16, 16, 16, 64, stream=0)
    t = B.spline_table_create(16, 16, 16, 64, coef)
    wisdom = str(tmp_path / "w.txt")
    try:
        best = B.spline_autotune(t, "vgh", 1024, wisdom)
        assert best.vw in (1, 2, 4) and best.wx * best.wy <= 8
        assert B.spline_tile_select(t, "vgh", 1024).as_tuple() == best.as_tuple()
        assert "single|" in open(wisdom).read()
        pos = synth.positions(1024, stream=1)
        from helpers import run_gpu
        gpu, _ = run_gpu(B, t, "vgh", pos, 64)  # tile=None -> the tuned one
        assert_close("vgh", gpu, oracle.evaluate("vgh", coef, pos), label="tuned")
    finally:
        B.spline_table_destroy(t)


CFG4 = [(32, 32, 32, 256), (40, 40, 40, 512), (48, 48, 48, 1152), (64, 64, 64, 2048)]
CFG4_NPOS = [97, 512, 1500, 3000]


@pytest.mark.parametrize("dtype,bound", [("f32", None), ("f16", 2e-3), ("bf16", 5e-3)])
def test_config4_batched_sampled(dtype, bound):
    """The four uneven tables of the batched workload in one launch replayed
    from the plan's graph, with the plan's autotuned tile (as the benchmark
    runs them); every position of the small table and 256 sampled positions
    of each other table are checked against the oracle: FP32 tables at 1e-5;
    FP16/BF16 tables at 1e-5 against the oracle on the dequantised
    coefficients and within their bound against the original ones."""
    dev = torch.device("cuda")
    handles, coefs = [], []
    try:
        for i, s in enumerate(CFG4):
            c = synth.coef_table(*s, stream=synth.table_stream(i))
            coefs.append(c)
            handles.append(B.spline_table_create(*s, c, dtype))
        pos = [synth.positions(n, stream=synth.position_stream(i))
               for i, n in enumerate(CFG4_NPOS)]
        pd = [torch.from_numpy(p).to(dev) for p in pos]
        ldo = [s[3] for s in CFG4]
        outs = [_outs("vgh", n, l) for n, l in zip(CFG4_NPOS, ldo)]
        plan = B.spline_batch_plan_create(handles, CFG4_NPOS, "vgh", pd,
                                          [o["v"] for o in outs], [o["g"] for o in outs],
                                          [o["h"] for o in outs], ldo, tile=None)
        B.spline_batch_execute(plan)
        B.spline_batch_execute(plan)
        torch.cuda.synchronize()
        rng = np.random.default_rng(4)
        for i in range(4):
            n = CFG4[i][3]
            idx = np.arange(CFG4_NPOS[i]) if CFG4_NPOS[i] <= 256 else \
                np.sort(rng.choice(CFG4_NPOS[i], 256, replace=False))
            got = {k: t.cpu().numpy()[idx][..., :n].astype(np.float64) for k, t in outs[i].items()}
            if dtype == "f32":
                assert_close("vgh", got, oracle.evaluate("vgh", coefs[i], pos[i][:, idx]),
                             label=f"config4 table {i}")
                continue
            assert_close("vgh", got, oracle.evaluate("vgh", dequantized(coefs[i], dtype),
                                                     pos[i][:, idx]),
                         label=f"config4 {dtype} table {i} vs dequantised")
            errs = normalized_errors("vgh", got, oracle.evaluate("vgh", coefs[i], pos[i][:, idx]))
            print(f"config4 {dtype} table {i}", {k: f"{e:.2e}" for k, e in errs.items()})
            assert max(errs.values()) <= bound, (i, errs)
        print("config4", dtype, "tile", B.spline_batch_plan_tile(plan))
        B.spline_batch_plan_destroy(plan)
    finally:
        for h in handles:
            B.spline_table_destroy(h)


@pytest.mark.parametrize("tile", [(1, 2, 1, 0, 0, 1), (2, 4, 1, 0, 1, 1), (4, 1, 2, 64, 2, 1),
                                  (1, 2, 2, 0, 4, 1)])
def test_batch_launch_matches_execute(tile):
    """spline_batch_launch issues the plan's kernels without the graph: the
    same bits as a graph replay, before and after a rebind, and inside a
    stream capture replayed several times with eager work in between."""
    shapes = [(6, 7, 5, 300), (5, 5, 6, 130), (7, 6, 6, 520)]
    npos = [77, 40, 150]
    coefs = [synth.coef_table(*s, stream=400 + i) for i, s in enumerate(shapes)]
    hs = [B.spline_table_create(*s, c, "f32") for s, c in zip(shapes, coefs)]
    dev = torch.device("cuda")

    def sets(stream0):
        pos = [torch.from_numpy(synth.positions(m, stream=stream0 + i) * 2 - 0.5).to(dev)
               for i, m in enumerate(npos)]
        outs = [_outs("vgh", m, s[3]) for m, s in zip(npos, shapes)]
        return pos, outs

    def host(outs):
        return [{k: t.cpu().numpy() for k, t in o.items()} for o in outs]

    try:
        pos, outs = sets(410)
        plan = B.spline_batch_plan_create(hs, npos, "vgh", pos, [o["v"] for o in outs],
                                          [o["g"] for o in outs], [o["h"] for o in outs],
                                          [s[3] for s in shapes], tile=tile)
        try:
            B.spline_batch_execute(plan)
            torch.cuda.synchronize()
            ref = host(outs)
            for o in outs:
                for t in o.values():
                    t.fill_(7.0)
            B.spline_batch_launch(plan)
            torch.cuda.synchronize()
            got = host(outs)
            for a, b in zip(ref, got):
                for k in a:
                    assert np.array_equal(a[k], b[k]), k
            # rebind table 1 to new buffers: launch sees it at once
            pos2, outs2 = sets(420)
            B.spline_batch_rebind(plan, 1, pos2[1], outs2[1]["v"], outs2[1]["g"], outs2[1]["h"])
            B.spline_batch_launch(plan)
            torch.cuda.synchronize()
            got2 = host(outs2)[1]
            ref2 = oracle.evaluate("vgh", coefs[1], pos2[1].cpu().numpy())
            assert_close("vgh", {k: a[..., :shapes[1][3]].astype(np.float64)
                                 for k, a in got2.items()}, ref2, label="launch after rebind")
            # captured into a caller's graph; each replay checked against the eager result
            B.spline_batch_rebind(plan, 1, pos[1], outs[1]["v"], outs[1]["g"], outs[1]["h"])
            gs = torch.cuda.Stream()
            gs.wait_stream(torch.cuda.current_stream())
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.stream(gs):
                B.spline_batch_launch(plan, gs.cuda_stream)
                torch.cuda.synchronize()
                with torch.cuda.graph(graph, stream=gs):
                    B.spline_batch_launch(plan, gs.cuda_stream)
            torch.cuda.synchronize()
            for _ in range(3):
                for o in outs:
                    for t in o.values():
                        t.fill_(3.0)
                torch.cuda.synchronize()
                graph.replay()
                torch.cuda.synchronize()
                for a, b in zip(ref, host(outs)):
                    for k in a:
                        assert np.array_equal(a[k], b[k]), ("replay", k)
            del graph
        finally:
            B.spline_batch_plan_destroy(plan)
    finally:
        for h in hs:
            B.spline_table_destroy(h)

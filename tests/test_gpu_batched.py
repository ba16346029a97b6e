"""GPU tests of the batched form (marked gpu).

Every product of a batch must equal the plain per-product call on the same
inputs bit for bit (and hence the oracle); graph replays are checked against
the eager result several times, with other work and synchronisations between.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev_mp, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    need_gpu()
    from paper_2609_27831_amd import oz2h
    return oz2h


def make_batch(seed, count, lo, hi, ps=(53, 113, 256, 512), elo=-4, ehi=4):
    """Log-uniform dimensions in [lo, hi], precision drawn from ps (the batched workload's recipe)."""
    u = synth.splitmix64(seed, 0, 4 * count).reshape(count, 4)
    out = []
    for i in range(count):
        f = (u[i, :3] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
        M, N, K = (int(round(lo * (hi / lo) ** x)) for x in f)
        p = ps[int(u[i, 3] % np.uint64(len(ps)))]
        A, B = synth.operands_for(seed * 1000 + i, M, N, K, p, elo, ehi)
        out.append((A, B))
    return out


def _host(C):
    s, e, l = C.to_host()
    return s, e, l


def test_batched_matches_plain_calls(oz, c_oracle):
    import torch
    batch = make_batch(7, 24, 16, 400)
    probs, devs = [], []
    for i, (A, B) in enumerate(batch):
        opA, opB = (i % 2, (i // 2) % 2)
        Ad = dev_mp(A.transpose() if opA else A)
        Bd = dev_mp(B.transpose() if opB else B)
        C = oz.empty_mp(A.shape[0], B.shape[1], A.p)
        probs.append((Ad, Bd, C, opA, opB))
    bp = oz.BatchedPlan(probs)
    ws = bp.workspace()
    print("batched eager", bp.config(), flush=True)
    bp.run_eager(ws)
    torch.cuda.synchronize()
    eager = [_host(C) for (_, _, C, _, _) in probs]
    for i, (Ad, Bd, C, opA, opB) in enumerate(probs):
        plan = oz.Plan.create(Ad.p, batch[i][0].shape[1])
        Cp = oz.gemm(plan, Ad, Bd, opA, opB)
        torch.cuda.synchronize()
        ref = _host(Cp)
        for a, b in zip(eager[i], ref):
            assert np.array_equal(a, b), f"product {i}"
    # the oracle on a few products
    for i in (0, 5, 11):
        A, B = batch[i]
        r = c_oracle.gemm(A, B, want_chat=False)
        s, e, l = eager[i]
        assert np.array_equal(s, r["c_sign"]) and np.array_equal(e, r["c_exp"])
        assert np.array_equal(l, r["c_limbs"])
    # graph replays, with other work between them
    for rep in range(3):
        for (_, _, C, _, _) in probs:
            C.sign.fill_(0)
            C.exp.fill_(0)
            C.limbs.fill_(0)
        torch.cuda.synchronize()
        print(f"batched graph replay {rep}", flush=True)
        bp.run(ws)
        torch.cuda.synchronize()
        for i, (_, _, C, _, _) in enumerate(probs):
            for a, b in zip(_host(C), eager[i]):
                assert np.array_equal(a, b), f"replay {rep} product {i}"
    bp.destroy()


@pytest.mark.parametrize("tile,bpc", [(1, 1), (2, 2), (3, 4), (2, 0), (0, 0), (0, 2)])
def test_batched_tiles_and_schedules(oz, tile, bpc):
    import torch
    batch = make_batch(11, 10, 100, 700, ps=(113, 512))
    probs = [(dev_mp(A), dev_mp(B), oz.empty_mp(A.shape[0], B.shape[1], A.p), 0, 0) for A, B in batch]
    bp = oz.BatchedPlan(probs, oz.default_opts(tile=tile))
    bp.set_config(tile, bpc)
    ws = bp.workspace()
    print(f"batched tile={tile} bpc={bpc}", bp.config(), flush=True)
    bp.run(ws)
    torch.cuda.synchronize()
    for i, (Ad, Bd, C, _, _) in enumerate(probs):
        Cp = oz.gemm(oz.Plan.create(Ad.p, Ad.shape[1]), Ad, Bd)
        torch.cuda.synchronize()
        for a, b in zip(_host(C), _host(Cp)):
            assert np.array_equal(a, b), f"product {i}"


@pytest.mark.parametrize("stages,graph", [(2, True), (2, False), (3, False)])
def test_batched_gemm_stages_and_run_mode(oz, stages, graph):
    """The two-stage grouped GEMM and the direct-launch mode of oz2h_batched_run give the
    plain calls' results bit for bit (two runs in a row, the second after a schedule change
    back and forth)."""
    import torch
    batch = make_batch(17, 10, 100, 700, ps=(53, 113, 512))
    probs = [(dev_mp(A), dev_mp(B), oz.empty_mp(A.shape[0], B.shape[1], A.p), 0, 0) for A, B in batch]
    bp = oz.BatchedPlan(probs)
    bp.set_schedule(stages, graph)
    cfg = bp.config()
    assert cfg["gemm_stages"] == stages and cfg["graph"] == graph
    ws = bp.workspace()
    print(f"batched stages={stages} graph={graph}", cfg, flush=True)
    ref = []
    for Ad, Bd, _, _, _ in probs:
        Cp = oz.gemm(oz.Plan.create(Ad.p, Ad.shape[1]), Ad, Bd)
        torch.cuda.synchronize()
        ref.append(_host(Cp))
    for rep in range(2):
        if rep:
            bp.set_schedule(5 - stages, not graph)
            bp.set_schedule(stages, graph)
        bp.run(ws)
        torch.cuda.synchronize()
        for i, (_, _, C, _, _) in enumerate(probs):
            for a, b in zip(_host(C), ref[i]):
                assert np.array_equal(a, b), f"run {rep} product {i}"
    with pytest.raises(oz.Oz2hError):
        bp.set_schedule(4, True)
    bp.destroy()


def test_batched_autotune(oz):
    import torch
    batch = make_batch(13, 8, 64, 512)
    probs = [(dev_mp(A), dev_mp(B), oz.empty_mp(A.shape[0], B.shape[1], A.p), 0, 0) for A, B in batch]
    bp = oz.BatchedPlan(probs)
    ws = bp.workspace()
    cfg = bp.tune(ws)
    print("tuned", cfg, flush=True)
    assert cfg["tile"] in (0, 1, 2, 3) and cfg["blocks_per_cu"] in (0, 1, 2, 4)
    assert cfg["gemm_stages"] in (2, 3)
    bp.run(ws)
    torch.cuda.synchronize()
    for i, (Ad, Bd, C, _, _) in enumerate(probs):
        Cp = oz.gemm(oz.Plan.create(Ad.p, Ad.shape[1]), Ad, Bd)
        torch.cuda.synchronize()
        for a, b in zip(_host(C), _host(Cp)):
            assert np.array_equal(a, b)
    # a second plan with the same shapes picks the tuned configuration up
    bp2 = oz.BatchedPlan(probs)
    c2 = bp2.config()
    assert c2["tile"] == cfg["tile"] and c2["blocks_per_cu"] == cfg["blocks_per_cu"]
    assert c2["gemm_stages"] == cfg["gemm_stages"] and c2["graph"] == cfg["graph"]


_TUNE_CHILD = r"""
import json, sys
import torch
sys.path.insert(0, sys.argv[1])
from paper_2609_27831_amd import oz2h
from tests.gpu_util import dev_mp
from tests.test_gpu_batched import make_batch
batch = make_batch(17, 4, 64, 256)
probs = [(dev_mp(A), dev_mp(B), oz2h.empty_mp(A.shape[0], B.shape[1], A.p), 0, 0) for A, B in batch]
bp = oz2h.BatchedPlan(probs)
cfg = bp.tune(bp.workspace()) if sys.argv[2] == "tune" else bp.config()
torch.cuda.synchronize()
print(json.dumps(cfg))
"""


def test_batched_tune_cache_file(oz, tmp_path):
    """OZ2H_TUNE_CACHE: a tuned configuration is appended as "signature tile bpc stages graph"
    and picked up by a new process; an older three-field line takes three stages and graph
    replay; lines that do not parse or hold out-of-range values are skipped.  Each step runs in
    a fresh process, since the library reads the file once per process."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, OZ2H_TUNE_CACHE=str(cache))

    def child(mode):
        print(f"tune-cache child: {mode}", flush=True)
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root, mode], cwd=root, env=env,
                           capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    tuned = child("tune")
    lines = cache.read_text().split()
    assert len(lines) == 5
    sig = lines[0]
    assert [int(x) for x in lines[1:]] == [tuned["tile"], tuned["blocks_per_cu"],
                                           tuned["gemm_stages"], int(tuned["graph"])]
    got = child("config")
    assert {k: got[k] for k in ("tile", "blocks_per_cu", "gemm_stages", "graph")} == \
        {k: tuned[k] for k in ("tile", "blocks_per_cu", "gemm_stages", "graph")}
    # later lines win; the three-field line is taken, the bad ones are skipped
    with open(cache, "a") as f:
        f.write(f"{sig} 1 0\n")
        f.write(f"{sig} 9 0 3 1\n")        # tile out of range
        f.write(f"{sig} 2 0 4 1\n")        # four LDS stages
        f.write(f"{sig} 2 99 3 0\n")       # blocks per CU out of range
        f.write("not a record\n")
    got = child("config")
    assert (got["tile"], got["blocks_per_cu"], got["gemm_stages"], got["graph"]) == (1, 0, 3, True)


def test_batched_full_workload(oz, c_oracle):
    """The full batched workload (64 products, M, N, K log-uniform in [128, 4096],
    p in {53, 113, 256, 512}, exponents U[-4, 4], the generator and seed the bench uses):
    graph replay bit-identical to the loop of plain calls, and every product against the
    oracle on sampled entries (its four corners plus seeded random ones)."""
    import time
    import torch
    t0 = time.time()
    seed = synth.CONFIG_SEED_BASE + 4
    u = synth.splitmix64(seed, 0, 4 * 64).reshape(64, 4)
    spec = []
    for i in range(64):
        f = (u[i, :3] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
        M, N, K = (int(round(128 * 32.0 ** x)) for x in f)
        spec.append((M, N, K, (53, 113, 256, 512)[int(u[i, 3] % np.uint64(4))], seed * 1000 + i))
    rng = np.random.default_rng(4)
    probs, samples = [], []
    for (M, N, K, p, sd) in spec:
        A, B = synth.operands_for(sd, M, N, K, p, -4, 4)
        si = np.array([0, 0, M - 1, M - 1] + list(rng.integers(0, M, 12)), np.int64)
        sj = np.array([0, N - 1, 0, N - 1] + list(rng.integers(0, N, 12)), np.int64)
        ref = c_oracle.gemm(A, B, sel=(si, sj), want_chat=False)
        samples.append((si, sj, ref))
        probs.append((dev_mp(A), dev_mp(B), oz.empty_mp(M, N, p), 0, 0))
        del A, B
    print(f"batched full workload: inputs and oracle samples {time.time() - t0:.1f}s", flush=True)
    bp = oz.BatchedPlan(probs)
    ws = bp.workspace()
    bp.tune(ws)
    bp.run(ws)
    torch.cuda.synchronize()
    got = [tuple(x.clone() for x in (C.sign, C.exp, C.limbs)) for (_, _, C, _, _) in probs]
    print(f"batched full workload: graph done {time.time() - t0:.1f}s {bp.config()}", flush=True)
    wsz = 256
    plans = []
    for (Ad, Bd, C, _, _) in probs:
        pl = oz.Plan.create(Ad.p, Ad.shape[1])
        plans.append(pl)
        wsz = max(wsz, pl.workspace_size(Ad.shape[0], Bd.shape[1]))
    ws1 = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    for i, (pl, (Ad, Bd, C, _, _)) in enumerate(zip(plans, probs)):
        Cp = oz.gemm(pl, Ad, Bd, ws=ws1)
        for a, b in zip(got[i], (Cp.sign, Cp.exp, Cp.limbs)):
            assert torch.equal(a, b), f"product {i}"
        si, sj, ref = samples[i]
        ti, tj = torch.from_numpy(si).cuda(), torch.from_numpy(sj).cuda()
        assert np.array_equal(got[i][0][ti, tj].cpu().numpy(), ref["c_sign"]), f"product {i}"
        assert np.array_equal(got[i][1][ti, tj].cpu().numpy(), ref["c_exp"]), f"product {i}"
        assert np.array_equal(got[i][2][ti, tj].cpu().numpy().view(np.uint64), ref["c_limbs"]), \
            f"product {i}"
    print(f"batched full workload: loop compared {time.time() - t0:.1f}s", flush=True)
    bp.destroy()

"""Batching and serving on the GPU (MI355X only).

Each request's result must be the same alone and in any batch or mix:
Jacobi has no atomics, so the bar is bit-exact -- against the single-grid
engine path run alone, and (within the 1e-6 stencil bar, expected exact)
against the oracle's in-order Jacobi program."""
import numpy as np
import pytest

from oracle import programs as OP
from paper_2012_08141_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


def _requests(count, lo=32, hi=600, iters=12, seed=3):
    from paper_2012_08141_amd.serving import Request
    reqs = []
    for i in range(count):
        w = I.batch_request(seed, i, n=128, lo=lo, hi=hi)
        reqs.append(Request(i, 0.0, w.cells, w.channels["b"], iters))
    return reqs


def test_batch_alone_equals_mix_and_oracle():
    """Requests admitted at different global iterations, advanced together by
    a captured graph, retired when done; every result equals the request run
    alone through the single-grid engine and the oracle."""
    from paper_2012_08141_amd.batching import BatchArena
    from paper_2012_08141_amd.serving import solve_alone
    say("batch mix")
    reqs = _requests(10)
    arena = BatchArena(128, max_grids=8, pool_blocks=4096)
    graph = arena.capture(5)
    results = {}
    pending = list(reqs)
    live = {}
    steps = 0
    while pending or live:
        # admit at most two per replay boundary, so grids overlap at offsets
        for _ in range(2):
            if pending and arena.fits(pending[0].nblocks):
                r = pending.pop(0)
                r.gid = arena.admit(r.cells, r.b, r.iters)
                r.end_clock = arena.clock_host + r.iters
                live[r.rid] = r
        for r in [r for r in live.values() if r.end_clock <= arena.clock_host]:
            results[r.rid] = arena.retire(r.gid)
            del live[r.rid]
        if live:
            graph.replay()
            steps += 1
    torch.cuda.synchronize()
    assert steps > 3
    for r in reqs:
        alone = solve_alone(r, 128, 0)
        got = results[r.rid].cpu().numpy()
        assert np.array_equal(got, alone.cpu().numpy()), r.rid
        ref = OP.jacobi_program(128, I.cells_to_blocks(r.cells, 16), r.b, r.iters)
        order = np.argsort(r.cells)          # cells are ascending already
        assert np.array_equal(ref["cells"], r.cells[order])
        exp = ref["x"]
        tol = 1e-6 * np.maximum(np.abs(exp), 1e-3 * np.abs(exp).max())
        assert np.all(np.abs(got - exp) <= tol), r.rid


def test_serving_continuous_batching():
    """A request stream through the server with a footprint budget that
    forces admission to wait: all requests finish, several are resident at
    once, and each result equals the request solved alone."""
    from paper_2012_08141_amd.serving import JacobiServer, solve_alone
    say("serving")
    reqs = _requests(12, lo=64, hi=1500, iters=20, seed=5)
    need = max(r.nblocks for r in reqs)
    budget = int(2.5 * need * (3 * 2048 + 4))
    srv = JacobiServer(128, budget_bytes=budget, max_grids=8, iters_per_replay=5)
    st = srv.serve(reqs, realtime=False)
    summ = st.summary()
    say("  ", summ)
    assert summ["requests"] == len(reqs)
    assert st.max_resident >= 2
    for r in reqs:
        assert r.completed >= 0 and r.result is not None
        assert np.array_equal(r.result.cpu().numpy(), solve_alone(r, 128, 0).cpu().numpy()), r.rid


def test_batch_graph_replays_match_eager_launches():
    """The captured graph gives the same state after every replay as direct
    launches (a HIP graph replayed several times, with host work between)."""
    from paper_2012_08141_amd.batching import BatchArena
    say("graph replays")
    reqs = _requests(4, iters=40)
    a1 = BatchArena(128, 4, 4096)
    a2 = BatchArena(128, 4, 4096)
    for r in reqs:
        a1.admit(r.cells, r.b, r.iters)
        a2.admit(r.cells, r.b, r.iters)
    g = a1.capture(4)
    for _ in range(6):
        g.replay()
        a2.step(4)
        torch.cuda.synchronize()
        assert torch.equal(a1.x, a2.x) and torch.equal(a1.xn, a2.xn)


@pytest.mark.parametrize("waves", [2, 4])
def test_batch_waves_per_workgroup_equal(waves):
    """Two or four wavefronts per workgroup give the same state as one."""
    from paper_2012_08141_amd.batching import BatchArena
    say("batch waves", waves)
    reqs = _requests(5, iters=30, seed=7)
    arenas = [BatchArena(128, 8, 4096), BatchArena(128, 8, 4096)]
    for a in arenas:
        for r in reqs:
            a.admit(r.cells, r.b, r.iters)
    g1 = arenas[0].capture(5, 512, 1)
    gw = arenas[1].capture(5, 512 // waves, waves)
    for _ in range(6):
        g1.replay()
        gw.replay()
    torch.cuda.synchronize()
    assert torch.equal(arenas[0].x, arenas[1].x) and torch.equal(arenas[0].xn, arenas[1].xn)


def test_autotuner_choice_is_a_candidate_and_correct():
    """The autotuner times every (waves, workgroups, iterations per replay)
    candidate and returns one of them; a graph captured with the choice
    gives the result of the default launch."""
    from paper_2012_08141_amd import autotune
    from paper_2012_08141_amd.batching import BatchArena
    say("autotune")
    reqs = _requests(4, iters=1 << 30, seed=9)
    scratch = BatchArena(128, 8, 4096)
    for r in reqs:
        scratch.admit(r.cells, r.b, r.iters)
    choice = autotune.tune_batch(scratch, "test", wavefronts=(1024, 2048), waves=(1, 2), iters=(2, 4),
                                 reps=2, use_cache=False)
    cands = {(c["waves"], c["workgroups"], c["iters_per_replay"]) for c in choice["candidates"]}
    assert len(cands) == 8
    assert (choice["waves"], choice["workgroups"], choice["iters_per_replay"]) in cands
    a1, a2 = BatchArena(128, 8, 4096), BatchArena(128, 8, 4096)
    for a in (a1, a2):
        for r in reqs[:2]:
            a.admit(r.cells, r.b, 12)
    K = choice["iters_per_replay"]
    g = a2.capture(K, choice["workgroups"], choice["waves"])
    done = 0
    while done < 12:
        g.replay()
        a1.step(K)
        done += K
    torch.cuda.synchronize()
    assert torch.equal(a1.x, a2.x)


def test_full_size_requests_alone_mix_and_oracle():
    """The serving workload at full size: the first 8 requests of the seed-0
    stream (100 to 3,107 blocks) and its largest (request 246, 4,083 blocks),
    50 iterations each, admitted at different replay boundaries of one
    captured graph.  Each result equals the request solved alone (bit for
    bit) and the oracle's in-order Jacobi program (within the stencil bar)."""
    from paper_2012_08141_amd.batching import BatchArena
    from paper_2012_08141_amd.serving import make_requests, solve_alone
    say("batch full-size requests")
    ids = list(range(8)) + [246]
    allr = make_requests(0, 247, np.zeros(247))
    reqs = [allr[i] for i in ids]
    assert max(r.nblocks for r in reqs) == 4083 and all(r.iters == 50 for r in reqs)
    arena = BatchArena(128, max_grids=16, pool_blocks=sum(r.nblocks for r in reqs))
    graph = arena.capture(5)
    pending, live, results = list(reqs), {}, {}
    while pending or live:
        if pending:                          # one admission per replay boundary
            r = pending.pop(0)
            r.gid = arena.admit(r.cells, r.b, r.iters)
            r.end_clock = arena.clock_host + r.iters
            live[r.rid] = r
        for r in [r for r in live.values() if r.end_clock <= arena.clock_host]:
            results[r.rid] = arena.retire(r.gid)
            del live[r.rid]
        if live:
            graph.replay()
    torch.cuda.synchronize()
    for r in reqs:
        say("  request", r.rid, r.nblocks, "blocks")
        got = results[r.rid].cpu().numpy()
        alone = solve_alone(r, 128, 0).cpu().numpy()
        assert np.array_equal(got, alone), r.rid
        ref = OP.jacobi_program(128, I.cells_to_blocks(r.cells, 16), r.b, r.iters)
        assert np.array_equal(ref["cells"], r.cells)
        exp = ref["x"]
        tol = 1e-6 * np.maximum(np.abs(exp), 1e-3 * np.abs(exp).max())
        assert np.all(np.abs(got - exp) <= tol), r.rid


def test_batch_update_validation_and_mixed_boundary():
    """at_batch_update rejects bad descriptors before enqueueing anything
    (the arena is unchanged afterwards), and one update that retires a grid
    and admits two others into its slots gives the results of separate
    calls: every result equals the request solved alone."""
    import ctypes
    from paper_2012_08141_amd import _lib as L
    from paper_2012_08141_amd.batching import BatchArena
    from paper_2012_08141_amd.grid import current_stream
    from paper_2012_08141_amd.serving import solve_alone
    say("batch update")
    reqs = _requests(3, lo=40, hi=300, iters=10, seed=11)
    pool = reqs[0].nblocks + max(reqs[1].nblocks + reqs[2].nblocks, 1)
    arena = BatchArena(128, max_grids=2, pool_blocks=pool)
    lib = L.lib()
    cells = torch.as_tensor(reqs[0].cells.astype(np.int32), device="cuda")
    b = torch.as_tensor(reqs[0].b, device="cuda")
    slots = torch.empty(len(reqs[0].cells), dtype=torch.int32, device="cuda")

    def adm(gid, nb=None, it=10, reserved=0):
        return L.AtBatchAdmit(cells.data_ptr(), b.data_ptr(), slots.data_ptr(), gid,
                              len(reqs[0].cells) if nb is None else nb, it, reserved)

    def call(rets, adms):
        ra = (L.AtBatchRetire * max(1, len(rets)))(*rets)
        aa = (L.AtBatchAdmit * max(1, len(adms)))(*adms)
        return lib.at_batch_update(arena.handle, ra, len(rets), aa, len(adms), current_stream())

    assert call([L.AtBatchRetire(0, 0, None)], []) == L.AT_E_INVALID          # not resident
    assert call([], [adm(2)]) == L.AT_E_INVALID                               # id out of range
    assert call([], [adm(0), adm(0)]) == L.AT_E_INVALID                       # same id twice
    assert call([], [adm(0, nb=0)]) == L.AT_E_INVALID                         # no blocks
    assert call([], [adm(0, it=-1)]) == L.AT_E_INVALID
    assert call([], [adm(0, reserved=1)]) == L.AT_E_INVALID
    assert call([], [adm(0, nb=pool + 1)]) == L.AT_E_INVALID
    assert call([], [adm(0), adm(1, nb=pool)]) == L.AT_E_CAPACITY
    torch.cuda.synchronize()
    assert int(arena.count.item()) == 0
    # request 0 alone, then one boundary retires it and admits 1 and 2
    g0 = arena.admit(reqs[0].cells, reqs[0].b, 10)
    for _ in range(2):
        arena.step(5)
    outs, gids = arena.update([g0], [(reqs[1].cells, reqs[1].b, 10), (reqs[2].cells, reqs[2].b, 10)])
    assert sorted(gids) == [0, 1]
    res = {0: outs[0]}
    for _ in range(2):
        arena.step(5)
    outs2, _ = arena.update(gids, [])
    res[1], res[2] = outs2
    torch.cuda.synchronize()
    assert int(arena.count.item()) == 0 and arena.free_blocks() == pool
    for i, r in enumerate(reqs):
        assert torch.equal(res[i], solve_alone(r, 128, 0)), i

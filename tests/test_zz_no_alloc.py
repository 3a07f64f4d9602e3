"""pilot_solve_static: the solve on the library's fixed device scratch.

Called through the C ABI, it must give pilot_solve's results bit for bit
(same kernels, same tiles), on two calls in a row with the second frame
smaller than the first, without allocating workspace (a context whose HBM
budget admits no workspace at all still solves), and refuse frames whose
workspace exceeds the scratch before launching anything."""
import numpy as np
import pytest
import torch

from synth import frames as S
from tests.gpu_common import say

pytestmark = pytest.mark.gpu

LEVELS = ((30, 40, 16), (60, 80, 32), (120, 160, 64))


def _frame(seed, N, M):
    return S.make_frame(2, 0, N=N, M=M, level_shapes=LEVELS, iters=(5, 5, 5), dsm_side=128, seed=seed)


def _tile_file(tmp_path, frames):
    """Gram-table variants for the middle level of each frame, the built-in
    heuristic elsewhere: both workspace layouts are exercised."""
    def lb(n):
        return max(int(n), 1).bit_length() - 1
    path = tmp_path / "tiles_static.txt"
    with open(path, "w") as fh:
        for f in frames:
            H, W, C = LEVELS[1]
            fh.write(f"C{C}_d0_N{lb(f.levels[1].N)}_M{lb(f.M)}_P{lb(H * W)}_v3 4 2 0 3\n")
    return str(path)


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("poses", "cost", "iterations", "status")) and a["best"] == b["best"]


def test_static_solve_equals_solve_on_two_calls(tmp_path):
    from paper_2606_31098_amd.pilot import Context, DeviceFrame, DeviceResult, PilotError
    fa, fb = _frame(41, N=900, M=21), _frame(42, N=350, M=6)          # the second call is smaller
    tiles = _tile_file(tmp_path, [fa, fb])
    da, db = DeviceFrame(fa), DeviceFrame(fb)
    ref = Context(0, tune_cache=tiles)
    ra, rb = ref.solve([da])[0], ref.solve([db])[0]
    torch.cuda.synchronize()
    ra, rb = ra.numpy(), rb.numpy()
    # a context whose HBM budget admits no workspace: pilot_solve cannot run,
    # pilot_solve_static does (it allocates nothing)
    ctx = Context(0, tune_cache=tiles, hbm_budget_bytes=4096)
    with pytest.raises(PilotError) as ei:
        ctx.solve([da])
    assert ei.value.code == -2, ei.value
    say("pilot_solve_static: frame A (N=900, M=21), then frame B (N=350, M=6)")
    sa = ctx.solve_static([da])[0]
    sb = ctx.solve_static([db])[0]
    torch.cuda.synchronize()
    sa, sb = sa.numpy(), sb.numpy()
    assert _same(sa, ra), "frame A: static solve differs from pilot_solve"
    assert _same(sb, rb), "frame B: static solve differs from pilot_solve"
    assert sb["status"].shape == (6,) and np.isfinite(sb["cost"]).all()
    # and again in the first order, on fresh result buffers: the scratch keeps
    # frame B's state, which must not leak into frame A's solve
    sa2 = ctx.solve_static([da], [DeviceResult(da.M)])[0]
    torch.cuda.synchronize()
    assert _same(sa2.numpy(), ra), "frame A after B: static solve differs from pilot_solve"
    ctx.close()
    ref.close()


def test_static_solve_of_a_batch_with_concurrent_launches(tmp_path):
    """Three frames whose tiles use different pass-kernel variants form three
    launch classes per pass, which run forked onto the context's side
    streams: the static solve of the batch equals pilot_solve's bit for bit."""
    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    fr = [_frame(51, N=900, M=21), _frame(52, N=500, M=9), _frame(53, N=700, M=40)]

    def lb(n):
        return max(int(n), 1).bit_length() - 1
    path = tmp_path / "tiles_batch.txt"
    with open(path, "w") as fh:
        for f, (variant, G) in zip(fr, ((3, 4), (4, 8), (1, 4))):
            for (H, W, C), L in zip(LEVELS, f.levels):
                fh.write(f"C{C}_d0_N{lb(L.N)}_M{lb(f.M)}_P{lb(H * W)}_v3 {G} 2 0 {variant}\n")
    dfs = [DeviceFrame(f) for f in fr]
    ref = Context(0, tune_cache=str(path))
    r = [x.numpy() for x in ref.solve(dfs)]
    ctx = Context(0, tune_cache=str(path), hbm_budget_bytes=4096)
    say("pilot_solve_static: a batch of three frames in three launch classes")
    s = [x.numpy() for x in ctx.solve_static(dfs)]
    torch.cuda.synchronize()
    for i in range(3):
        assert _same(s[i], r[i]), i
    ctx.close()
    ref.close()


def test_static_solve_at_the_benchmark_size():
    """The benchmark's workload (1 frame, N = 16384, M = 1024, bf16 pyramid
    up to 480x640x128, the committed tile database, anchors sorted, packed
    tiles) fits the fixed scratch and solves bitwise as pilot_solve does."""
    import os
    from paper_2606_31098_amd.pilot import Context, DeviceFrame
    tiles = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_31098_amd",
                         "tiles_gfx950.txt")
    f = S.make_frame(3, 0)
    d = DeviceFrame(f, dtype="bf16")
    ref = Context(0, tune_cache=tiles)
    r = ref.solve([d])[0]
    torch.cuda.synchronize()
    r = r.numpy()
    ctx = Context(0, tune_cache=tiles, hbm_budget_bytes=4096)
    say("pilot_solve_static: the 16384 x 1024 bf16 frame")
    s = ctx.solve_static([d])[0]
    torch.cuda.synchronize()
    assert _same(s.numpy(), r), "static solve differs from pilot_solve at the benchmark size"
    ctx.close()
    ref.close()


def test_static_solve_refuses_frames_beyond_the_scratch():
    from paper_2606_31098_amd.pilot import Context, DeviceFrame, DeviceResult, PilotError
    # 65536 hypotheses over 8192 anchors: about 110 MB of LM states and
    # partial sums, more than the 64 MiB scratch
    f = S.make_frame(2, 0, N=8192, M=1, level_shapes=((30, 40, 16),), iters=(2,), dsm_side=128, seed=43)
    f.poses = np.repeat(f.poses[:1], 65536, axis=0)
    d = DeviceFrame(f)
    res = DeviceResult(d.M)
    res.cost.fill_(-7.0)
    ctx = Context(0)
    with pytest.raises(PilotError) as ei:
        ctx.solve_static([d], [res])
    assert ei.value.code == -2 and "scratch" in str(ei.value), ei.value
    torch.cuda.synchronize()
    assert bool((res.cost == -7.0).all())                  # nothing was launched
    ctx.close()

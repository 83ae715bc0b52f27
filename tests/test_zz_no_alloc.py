"""GPU test of nlrmm_backproject_noalloc, the backprojection that allocates nothing: through
the C ABI it returns the same images as nlrmm_backproject (bitwise: same view split) and
matches the FP64 oracle, on two calls in a row with the second on a smaller input; it runs
under HIP graph capture on a context whose workspace was never grown (where growing a
workspace is refused), replaying equal to the eager result; a shape whose view split needs
more than the fixed scratch is refused on the host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import projector as P  # noqa: E402
from paper_2605_06336_amd import _lib, ops, synth  # noqa: E402

TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def case(N, nb, V, ncols, seed):
    th = synth.random_angles(V, seed)
    y = synth.random_sinogram(V * ncols, nb, seed=seed + 1).reshape(ncols, V, nb)
    return th, y.astype(np.float32)


def call(fn_name, ctx, g, V, ncols, yt, tht, out):
    b = ops.single(V)
    lib = _lib.lib()
    rc = getattr(lib, fn_name)(ctx, ctypes.byref(g), ctypes.byref(b), ncols, yt.data_ptr(),
                               tht.data_ptr(), out.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    return rc


def test_noalloc_matches_backproject_on_two_calls():
    ctx = ops.context(0)
    # 256^2 / 360 views uses a 16-way view split (partial images in the scratch); the second
    # call is smaller (128^2, 97 views, one column) and reuses the scratch the first one left
    for N, nb, V, ncols, seed in [(256, 363, 360, 2, 31), (128, 181, 97, 1, 41)]:
        g = ops.geom(N, nb)
        th, y = case(N, nb, V, ncols, seed)
        tht = torch.as_tensor(th, device="cuda")
        yt = torch.as_tensor(y, device="cuda")
        x_na = torch.full((ncols, 1, N, N), float("nan"), dtype=torch.float32, device="cuda")
        x_ref = torch.empty_like(x_na)
        print(f"noalloc backprojection {N}x{N}, {V} views, {ncols} columns", flush=True)
        assert call("nlrmm_backproject_noalloc", ctx, g, V, ncols, yt, tht, x_na) == 0
        assert call("nlrmm_backproject", ctx, g, V, ncols, yt, tht, x_ref) == 0
        torch.cuda.synchronize()
        a, r = x_na.cpu().numpy(), x_ref.cpu().numpy()
        assert np.array_equal(a, r)
        x_ora = P.backproject(y.astype(np.float64), th, N).reshape(a.shape)
        assert rel(a, x_ora) <= TOL, rel(a, x_ora)


def test_noalloc_under_graph_capture_on_a_fresh_context():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    assert lib.nlrmm_ctx_create(ctypes.byref(h), 0) == 0
    ctx = h.value
    try:
        N, nb, V, ncols = 256, 363, 360, 1
        g = ops.geom(N, nb)
        th, y = case(N, nb, V, ncols, 51)
        tht = torch.as_tensor(th, device="cuda")
        yt = torch.as_tensor(y, device="cuda")
        x_eager = torch.empty((ncols, 1, N, N), dtype=torch.float32, device="cuda")
        x_graph = torch.zeros_like(x_eager)
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        print("capturing nlrmm_backproject_noalloc on a fresh context", flush=True)
        with torch.cuda.graph(graph):
            rc = call("nlrmm_backproject_noalloc", ctx, g, V, ncols, yt, tht, x_graph)
        assert rc == 0
        assert call("nlrmm_backproject_noalloc", ctx, g, V, ncols, yt, tht, x_eager) == 0
        torch.cuda.synchronize()
        ref = x_eager.cpu().numpy()
        for rep in range(3):
            x_graph.zero_()
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(x_graph.cpu().numpy(), ref), rep
            # eager work on the same scratch between replays
            assert call("nlrmm_backproject_noalloc", ctx, g, V, ncols, yt, tht, x_eager) == 0
            torch.cuda.synchronize()
        x_ora = P.backproject(y.astype(np.float64), th, N).reshape(ref.shape)
        assert rel(ref, x_ora) <= TOL
        del graph
    finally:
        torch.cuda.synchronize()
        lib.nlrmm_ctx_destroy(ctx)


def test_noalloc_refuses_a_split_larger_than_the_scratch(tmp_path):
    ctx = ops.context(0)
    N, nb, V, ncols = 256, 363, 360, 20
    g = ops.geom(N, nb)
    # a stored 16-way split for 20 columns needs 16 x 20 x 256 KiB = 80 MiB of partial images
    path = str(tmp_path / "tune.txt")
    with open(path, "w") as f:
        f.write(f"1 {N} {N} {nb} 1 {ncols} {V} 16\n")
    ops.set_tune_file(path)
    try:
        th, y = case(N, nb, V, 1, 61)
        tht = torch.as_tensor(th, device="cuda")
        yt = torch.zeros((ncols, V, nb), dtype=torch.float32, device="cuda")
        x = torch.full((ncols, 1, N, N), 7.0, dtype=torch.float32, device="cuda")
        assert call("nlrmm_backproject_noalloc", ctx, g, V, ncols, yt, tht, x) == -2
        torch.cuda.synchronize()
        assert bool((x == 7.0).all())   # nothing was launched
    finally:
        ops.set_tune_file(None)

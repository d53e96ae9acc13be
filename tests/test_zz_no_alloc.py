"""The allocation-free closest-hit call against pt_trace_closest, through the C ABI.

Both calls run the same BVH walk (Sec. 5.1.1: closest hit through boxes
grouped so that every child lies inside its parent); the allocation-free one
keeps its stack spill and counters in the library's static device array and
may run a smaller grid.  Hits must agree bit for bit (ids, t, b1, b2), on two
calls in a row, the second with fewer rays, for a one-level and a two-level
hierarchy.
"""
import numpy as np
import pytest

from paper_2407_19977_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2407_19977_amd import pt
    return pt


def _rays(sc, n, seed, tmin):
    """Half from random points of a box around the scene in random directions,
    half from the camera towards its look-at point with a spread."""
    r = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.array([-30.0, 0.0, -30.0]), np.array([30.0, 5.0, 30.0])
    h = n // 2
    o = np.concatenate([r.uniform(lo, hi, size=(h, 3)), np.tile(np.array(sc.camera.eye, np.float64), (n - h, 1))])
    d = r.normal(size=(n, 3))
    d[h:] = np.array(sc.camera.look_at) - np.array(sc.camera.eye) + r.normal(size=(n - h, 3)) * 8.0
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = tmin
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


@pytest.mark.parametrize("which", ["spheres", "instanced"])
def test_noalloc_trace_equals_trace_closest(P, which):
    sc = scenes.spheres() if which == "spheres" else scenes.instanced()
    s = P.scene_from(sc, device=0)
    try:
        for call, n in enumerate(((1 << 21) + 77, 1000)):
            _say(f"[noalloc] {which}: call {call}, {n} rays")
            rays = _rays(sc, n, 40 + call, 1e-4)
            rd = torch.from_numpy(rays).to("cuda:0")
            h_ref = torch.empty((n, 6), dtype=torch.int32, device="cuda:0")
            h_new = torch.full((n, 6), -7, dtype=torch.int32, device="cuda:0")
            s.trace_closest(rd, h_ref)
            s.trace_closest_noalloc(rd, h_new)
            a = h_ref.cpu().numpy().view(np.uint32)
            b = h_new.cpu().numpy().view(np.uint32)
            assert a[:, 5].sum() > n // 8, "too few rays hit to tell anything"
            bad = np.argwhere((a != b).any(1))
            assert len(bad) == 0, f"{len(bad)} rays differ, first {bad[:5].ravel()}"
        # brute force needs no scratch; the call still answers it
        n = 333
        rays = _rays(sc, n, 50, 1e-4)
        rd = torch.from_numpy(rays).to("cuda:0")
        h_ref = torch.empty((n, 6), dtype=torch.int32, device="cuda:0")
        h_new = torch.empty_like(h_ref)
        s.trace_closest(rd, h_ref, brute_force=True)
        s.trace_closest_noalloc(rd, h_new, brute_force=True)
        assert torch.equal(h_ref, h_new)
    finally:
        s.close()


def test_noalloc_trace_argument_errors(P):
    sc = scenes.cornell()
    s = P.scene_from(sc, device=0)
    try:
        rd = torch.zeros((4, 8), dtype=torch.float32, device="cuda:0")
        h = torch.empty((4, 6), dtype=torch.int32, device="cuda:0")
        assert P.lib().pt_trace_closest_noalloc(s.h, rd.data_ptr(), -1, h.data_ptr(), 0) == -1
        assert P.lib().pt_trace_closest_noalloc(s.h, None, 4, h.data_ptr(), 0) == -1
        assert P.lib().pt_trace_closest_noalloc(s.h, rd.data_ptr(), 0, h.data_ptr(), 0) == 0
    finally:
        s.close()

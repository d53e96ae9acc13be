"""GPU parity of the display path (Sec. 5.1.4: the running mean is tone mapped
with Khronos PBR Neutral and shown after every sampling iteration) against
the FP64 oracle, through the C ABI.

Both sides compute in FP64 from the same FP64 sums, so the 8-bit codes agree
bit for bit, except where 255 e + 1/2 lies within 1e-9 of an integer (the
two sides' pow() may differ in the last bit): there a code may differ by
one.  The encoded values (FP64 rounded to float) agree within one float ulp.
The sums come from the seeded generator of the display inputs, loaded with
pt_set_accumulation; a progressive render is then checked against the
oracle's own render and display.
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


@pytest.fixture(scope="module")
def box(P):
    sc = scenes.cornell()
    s = P.scene_from(sc, device=0)
    yield sc, s
    s.close()


def _gpu_display(s, sums, samples, exposure):
    h, w = sums.shape[:2]
    s.set_accumulation(torch.from_numpy(np.ascontiguousarray(sums)).to("cuda:0"), samples)
    rgba = torch.zeros((h, w, 4), dtype=torch.uint8, device="cuda:0")
    enc = torch.zeros((h, w, 3), dtype=torch.float32, device="cuda:0")
    s.display(rgba, enc, exposure)
    return rgba.cpu().numpy(), enc.cpu().numpy()


def _check(O, sums, samples, exposure, g_rgba, g_enc, what):
    ref_enc, ref_rgba = O.display(sums, samples, exposure)
    assert np.all(g_rgba[..., 3] == 255)
    frac = 255.0 * ref_enc + 0.5
    near = np.abs(frac - np.round(frac)) < 1e-9
    diff = g_rgba[..., :3].astype(np.int32) - ref_rgba[..., :3].astype(np.int32)
    _say(f"[display] {what}: {sums.shape[1]}x{sums.shape[0]}, {np.count_nonzero(diff)} codes differ "
         f"({np.count_nonzero(near)} near a code boundary)")
    assert np.all(diff[~near] == 0), np.argwhere((diff != 0) & ~near)[:5]
    assert np.all(np.abs(diff[near]) <= 1)
    ref32 = ref_enc.astype(np.float32)
    ulp = np.spacing(np.maximum(np.abs(ref32), np.float32(1e-38)))
    assert np.all(np.abs(g_enc - ref32) <= ulp), np.abs(g_enc - ref32).max()
    # every branch of the tone map and of the transfer function was exercised
    assert (ref_rgba[..., :3] == 0).any() and (ref_rgba[..., :3] == 255).any()
    return ref_rgba


@pytest.mark.parametrize("w,h,samples,exposure", [(1920, 1080, 64, 1.0), (37, 23, 3, 2.5), (1, 1, 1, 1.0),
                                                  (1, 7, 5, 0.0)])
def test_display_matches_oracle(P, O, box, w, h, samples, exposure):
    _, s = box
    sums = scenes.display_sums(w, h, samples, seed=w + h)
    if w * h == 1:
        sums[0, 0] = [0.5, 80.0, 0.0]
    g_rgba, g_enc = _gpu_display(s, sums, samples, exposure)
    if exposure == 0.0:
        assert np.all(g_rgba[..., :3] == 0) and np.all(g_enc == 0.0)
        return
    if w * h == 1:
        ref_enc, ref_rgba = O.display(sums, samples, exposure)
        assert np.array_equal(g_rgba, ref_rgba)
        return
    _check(O, sums, samples, exposure, g_rgba, g_enc, f"synthetic sums, exposure {exposure}")


def test_progressive_display_follows_the_running_mean(P, O, box):
    """Display after every pt_accumulate (1 + 3 + 12 samples of the closed box):
    the image of the GPU's sums is the display of those sums (bitwise, reloaded
    through pt_set_accumulation) and agrees with the oracle's own render and
    display of the same samples up to the per-path tolerance (a few codes off by one)."""
    sc, s = box
    cam, depth = sc.camera, sc.max_depth
    W, H = cam.width, cam.height
    s.reset_accumulation()
    os_ = O.OracleScene(sc)
    done = 0
    for n in (1, 3, 12):
        s.accumulate(cam, done, n, depth, 0)
        done += n
        rgba = torch.zeros((H, W, 4), dtype=torch.uint8, device="cuda:0")
        s.display(rgba)
        out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda:0")
        sums = torch.empty((H, W, 3), dtype=torch.float64, device="cuda:0")
        s.resolve(out, sums)
        a = rgba.cpu().numpy()
        g2, _ = _gpu_display(s, sums.cpu().numpy(), done, 1.0)
        assert np.array_equal(a, g2)
        ref_sum = os_.render(done, depth, n_threads=16)["sum"]
        _, ref_rgba = O.display(ref_sum, done, 1.0)
        d = np.abs(a[..., :3].astype(np.int32) - ref_rgba[..., :3].astype(np.int32))
        _say(f"[display] progressive at {done} spp: {np.count_nonzero(d)} of {d.size} codes differ, max {d.max()}")
        # a pixel holding a path whose events left the oracle's (well under 1 % of pixels) may
        # differ by more than one code; elsewhere the sums agree to the per-path tolerance
        px = d.max(-1)
        assert np.count_nonzero(px) <= 0.03 * px.size and np.count_nonzero(px > 1) <= 0.01 * px.size
        s.set_accumulation(sums, done)  # continue from the same sums


def test_display_errors(P, box):
    sc, _ = box
    s = P.scene_from(sc, device=0)
    try:
        rgba = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda:0")
        lib = P.lib()
        assert lib.pt_display(s.h, 1.0, rgba.data_ptr(), None) == -5  # nothing accumulated
        sums = torch.ones((4, 4, 3), dtype=torch.float64, device="cuda:0")
        assert lib.pt_set_accumulation(s.h, sums.data_ptr(), 4, 4, 0) == -1
        assert lib.pt_set_accumulation(s.h, None, 4, 4, 1) == -1
        s.set_accumulation(sums, 2)
        assert lib.pt_display(s.h, 1.0, None, None) == -1
        assert lib.pt_display(s.h, -1.0, rgba.data_ptr(), None) == -1
        assert lib.pt_display(s.h, float("nan"), rgba.data_ptr(), None) == -1
        assert lib.pt_display(s.h, 1.0, rgba.data_ptr(), None) == 0
    finally:
        s.close()

"""GPU BVH construction (the paper times its CPU BVH set-up as a stage of its
own, Sec. 5.1.1, Table 1) against the host builder and the definition of the
closest hit, through the C ABI.

Both device builders (locally-ordered clustering, the default, and the
linear BVH) are checked.  Any valid tree is acceptable: what must hold is (a) the BVH4 invariants
(leaves partition the triangles, at most 4 per leaf, every child box inside
its parent's box of it, the reported depth), (b) closest hits bit-exact
against brute force and against the host-built tree on the same rays, and
(c) renders bitwise equal to those through the host-built tree (same hits,
same shading, same sums).
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


def _fields(nodes):
    f = nodes.view(np.float32).reshape(-1, 32)
    u = nodes.view(np.uint32).reshape(-1, 32)
    lo = np.stack([f[:, 0:4], f[:, 8:12], f[:, 16:20]], -1)   # [n, 4, 3]
    hi = np.stack([f[:, 4:8], f[:, 12:16], f[:, 20:24]], -1)
    return lo, hi, u[:, 24:28], u[:, 28]


def check_bvh4(nodes, tris, roots, tri_ranges):
    """BVH4 invariants of the trees rooted at `roots` whose triangles are `tri_ranges`."""
    lo, hi, child, nkids = _fields(nodes)
    tv = tris.view(np.float32).reshape(-1, 12)
    covered = np.zeros(len(tris), np.int32)
    depth_max = 0
    for root, (t0, t1) in zip(roots, tri_ranges):
        stack = [(root, 1)]
        while stack:
            k, d = stack.pop()
            assert 1 <= nkids[k] <= 4
            for c in range(4):
                r = int(child[k, c])
                if c >= nkids[k]:
                    assert r == 0xFFFFFFFF
                    continue
                if r & 0x80000000:
                    cnt, first = (r >> 27) & 7, r & ((1 << 27) - 1)
                    assert 1 <= cnt <= 4 and t0 <= first and first + cnt <= t1
                    covered[first:first + cnt] += 1
                    v = tv[first:first + cnt][:, [0, 1, 2, 4, 5, 6, 8, 9, 10]].reshape(-1, 3, 3)
                    assert np.all(v >= lo[k, c] - 0.0) and np.all(v <= hi[k, c] + 0.0), (k, c)
                    depth_max = max(depth_max, d + 1)
                else:
                    assert r < len(nodes)
                    n_kids = nkids[r]
                    assert np.all(lo[r, :n_kids] >= lo[k, c]) and np.all(hi[r, :n_kids] <= hi[k, c]), (k, c)
                    stack.append((r, d + 1))
    assert np.all(covered == 1), "every triangle in exactly one leaf"
    return depth_max


def _rays(n, seed, lo, hi, eye, look, tmin, spread):
    r = np.random.Generator(np.random.PCG64(seed))
    h = n // 2
    o = np.concatenate([r.uniform(lo, hi, size=(h, 3)), np.tile(np.array(eye, np.float64), (n - h, 1))])
    d = r.normal(size=(n, 3))
    d[h:] = np.array(look) - np.array(eye) + r.normal(size=(n - h, 3)) * spread
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = tmin
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


CASES = {
    "cornell": (scenes.cornell, (0, 0, 0), (1, 1, 1), 0.3),
    "zoo": (scenes.material_zoo, (0, 0, 0), (1, 1, 1), 0.3),
    "spheres": (scenes.spheres, (-13, 0, -13), (13, 3, 13), 6.0),
    "instanced": (scenes.instanced, (-30, 0, -30), (30, 5, 30), 12.0),
}


BUILDERS = ["ploc", "lbvh"]


@pytest.mark.parametrize("builder", BUILDERS)
@pytest.mark.parametrize("which", list(CASES))
def test_gpu_bvh_valid_and_hits_bit_exact(P, which, builder):
    make, lo, hi, spread = CASES[which]
    sc = make()
    s_gpu = P.scene_from(sc, device=0, gpu_bvh=builder)
    s_cpu = P.scene_from(sc, device=0)
    try:
        gi, ci = s_gpu.bvh_info(), s_cpu.bvh_info()
        _say(f"[gpu bvh] {which} ({builder}): {gi['n_tris']} triangles, device build {gi['build_ms']:.1f} ms "
             f"({gi['n_nodes']} nodes, depth {gi['depth']}), host build {ci['build_ms']:.1f} ms "
             f"({ci['n_nodes']} nodes, depth {ci['depth']})")
        assert gi["n_tris"] == ci["n_tris"] and gi["max_leaf_tris"] <= 4
        nodes, tris = s_gpu.copy_bvh()
        if sc.instances:
            # the meshes' trees are concatenated: roots and triangle ranges per mesh
            sizes = [m.n_triangles for m in sc.meshes]
            starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
            lo_, hi_, child, nk = _fields(nodes)
            # a mesh's root is the first node appended for it: find them by walking from node 0
            roots, k = [], 0
            for m, n_t in enumerate(sizes):
                roots.append(k)
                sub = [k]
                seen = 0
                while sub:
                    q = sub.pop()
                    seen += 1
                    for c in range(nk[q]):
                        r = int(child[q, c])
                        if not r & 0x80000000:
                            sub.append(r)
                k += seen
            depth = check_bvh4(nodes, tris, roots, [(a, a + b) for a, b in zip(starts, sizes)])
        else:
            depth = check_bvh4(nodes, tris, [0], [(0, len(tris))])
            assert depth == gi["depth"]
            # triangle records: the original triangles, each once
            prim = tris.view(np.uint32).reshape(-1, 12)[:, 3]
            assert np.array_equal(np.sort(prim), np.arange(len(tris)))
        n = 1 << 16
        rays = _rays(n, 60, lo, hi, sc.camera.eye, sc.camera.look_at, 1e-4, spread)
        rd = torch.from_numpy(rays).to("cuda:0")
        h_gpu = torch.empty((n, 6), dtype=torch.int32, device="cuda:0")
        h_cpu = torch.empty_like(h_gpu)
        h_bf = torch.empty_like(h_gpu)
        s_gpu.trace_closest(rd, h_gpu)
        s_cpu.trace_closest(rd, h_cpu)
        s_gpu.trace_closest(rd, h_bf, brute_force=True) if which in ("cornell", "zoo") else None
        a, b = h_gpu.cpu().numpy(), h_cpu.cpu().numpy()
        assert a[:, 5].sum() > n // 8
        bad = np.argwhere((a != b).any(1)).ravel()
        assert len(bad) == 0, f"{len(bad)} rays differ from the host-built tree, first {bad[:5]}"
        if which in ("cornell", "zoo"):
            assert np.array_equal(a, h_bf.cpu().numpy())
    finally:
        s_gpu.close()
        s_cpu.close()


def test_gpu_bvh_render_equals_host_bvh_render(P):
    """Same hits, same shading, same FP64 sums: the images are bitwise equal."""
    sc = scenes.material_zoo(width=64, height=64)
    outs = []
    for gpu in (False, "ploc", "lbvh"):
        s = P.scene_from(sc, device=0, gpu_bvh=gpu)
        out = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda:0")
        s.render(sc.camera, 8, 6, 0, out)
        outs.append(out.cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("builder", BUILDERS)
@pytest.mark.parametrize("n_tris", [1, 2, 4, 5, 17, 1000])
def test_gpu_bvh_small_and_degenerate_meshes(P, n_tris, builder):
    """Few triangles (a one-leaf root up to 4), and all centroids in one Morton
    cell (equal codes, ties broken by the index; for the clustering, equal
    boxes: every merged box has the same area, and the ties pair neighbours)."""
    r = np.random.Generator(np.random.PCG64(n_tris))
    for same_cell in (False, True):
        c = np.zeros((n_tris, 1, 3)) if same_cell else r.uniform(-1, 1, (n_tris, 1, 3))
        v = (c + 0.05 * r.normal(size=(n_tris, 3, 3))).reshape(-1, 3).astype(np.float32)
        if same_cell:  # equal centroids: every triangle is a permutation of the same three points
            base = r.normal(size=(3, 3)) * 0.05
            v = np.concatenate([base[np.roll(np.arange(3), k)] for k in range(n_tris)]).astype(np.float32)
        mesh = scenes.Mesh(v, np.arange(3 * n_tris, dtype=np.int32).reshape(-1, 3), np.zeros(n_tris, np.int32))
        s = P.PtScene(0)
        try:
            s.set_gpu_bvh_builder(builder)
            s.build_bvh([mesh], on_device=True)
            info = s.bvh_info()
            nodes, tris = s.copy_bvh()
            depth = check_bvh4(nodes, tris, [0], [(0, n_tris)])
            assert depth == info["depth"] and info["n_nodes"] == len(nodes)
            if n_tris <= 4:
                assert info["n_nodes"] == 1 and info["depth"] == 2
            s.upload_materials(scenes.lambert((0.5, 0.5, 0.5))[None, :])
            rays = _rays(4096, 70 + n_tris, (-1.5, -1.5, -1.5), (1.5, 1.5, 1.5), (0, 0, -3), (0, 0, 0), 1e-6, 0.3)
            rd = torch.from_numpy(rays).to("cuda:0")
            hb = torch.empty((4096, 6), dtype=torch.int32, device="cuda:0")
            hf = torch.empty_like(hb)
            s.trace_closest(rd, hb)
            s.trace_closest(rd, hf, brute_force=True)
            assert torch.equal(hb, hf)
        finally:
            s.close()


def test_gpu_bvh_builder_choice_is_checked(P):
    s = P.PtScene(0)
    try:
        for bad in ("sah", ""):
            with pytest.raises(P.PtError) as e:
                s.set_gpu_bvh_builder(bad)
            assert e.value.status == -1
    finally:
        s.close()

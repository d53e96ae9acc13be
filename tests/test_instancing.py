"""Two-level hierarchy (CPU): instanced scenes.

* The oracle's instancing is pinned against the same geometry flattened into
  world space: with rotations by multiples of 90 degrees and integer
  translations every transformed vertex is exact, so both must find the same
  closest triangles at the same distances.
* The library's two-level walk (compiled for the CPU) returns bit for bit the
  closest hits of the oracle's single-precision brute force over all
  instances: the ray enters object space in the fixed FP32 order and t is
  compared in each instance's object space.
* The instanced scene generator keeps its invariants (closed, outward meshes,
  triangle budgets, no overlapping instances, material mix).
"""
import numpy as np
import pytest

from paper_2407_19977_amd import scenes


def _small_meshes():
    v1, f1 = scenes.icosphere(2)
    v2, f2 = scenes.torus(0.7, 0.25, 24, 12)
    v3, f3 = scenes.bevelled_cylinder(0.6, 1.0, 0.1, 20, 4, 5)
    out = []
    for v, f in ((v1 * 0.8, f1), (v2, f2), (v3, f3)):
        v = np.round(v * 1024.0) / 1024.0  # coarse grid: integer translations stay exact in float
        out.append(scenes.Mesh(v.astype(np.float32), f.astype(np.int32), np.zeros(len(f), np.int32)))
    return out


def _rot90(rng):
    """A random signed permutation matrix with determinant +1 (exact rotation)."""
    while True:
        P = np.eye(3)[rng.permutation(3)] * rng.choice([-1.0, 1.0], size=(3, 1))
        if np.linalg.det(P) > 0:
            return P


def _scene(meshes, exact, n=24, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    insts = []
    for k in range(n):
        R = _rot90(rng) if exact else scenes._shoemake(*rng.uniform(size=3))
        t = np.array([3.0 * (k % 6) - 7.0, float(rng.integers(0, 3)), 3.0 * (k // 6) - 4.0])
        if not exact:
            t = t + rng.uniform(-0.3, 0.3, 3)
        M = np.hstack([R, t[:, None]]).astype(np.float32)
        insts.append(scenes.Instance(M, int(rng.integers(0, len(meshes))), 0))
    cam = scenes.Camera((0, 5, -15), (0, 0, 0), (0, 1, 0), 50.0, 8, 8)
    return scenes.Scene("inst", meshes, insts, np.stack([scenes.lambert((0.5, 0.5, 0.5))]), None, cam, 1, 1)


def _flatten(sc):
    verts, idx, prim_of = [], [], []
    base = 0
    for i, ins in enumerate(sc.instances):
        m = sc.meshes[ins.mesh]
        M = ins.object_to_world.astype(np.float64)
        v = m.vertices.astype(np.float64) @ M[:, :3].T + M[:, 3]
        verts.append(v)
        idx.append(m.indices + base)
        prim_of += [(i, p) for p in range(m.n_triangles)]
        base += len(v)
    v = np.concatenate(verts)
    assert np.array_equal(v.astype(np.float32).astype(np.float64), v)  # exact transforms
    mesh = scenes.Mesh(v.astype(np.float32), np.concatenate(idx).astype(np.int32),
                       np.zeros(sum(len(x) for x in idx), np.int32))
    flat = scenes.Scene("flat", [mesh], [], sc.materials, None, sc.camera, 1, 1)
    return flat, prim_of


def _rays(n, seed, lo=(-9, -2, -6), hi=(9, 4, 9)):
    r = np.random.Generator(np.random.PCG64(seed))
    o = r.uniform(lo, hi, size=(n, 3))
    d = r.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o, d


def test_oracle_instancing_matches_flattened_geometry(O):
    sc = _scene(_small_meshes(), exact=True)
    flat, prim_of = _flatten(sc)
    oi, of = O.OracleScene(sc), O.OracleScene(flat)
    o, d = _rays(3000, 1)
    agree = hits = 0
    for k in range(len(o)):
        a = oi.closest(o[k], d[k], tmin=1e-4)
        b = of.closest(o[k], d[k], tmin=1e-4)
        assert a[0] == b[0]
        if not a[0]:
            agree += 1
            continue
        hits += 1
        if (a[4], a[5]) == prim_of[b[5]] and abs(a[1] - b[1]) <= 1e-9 * b[1]:
            agree += 1
    assert hits > 300
    assert agree >= len(o) - 3


def _rays_f32(sc, n, seed):
    o, d = _rays(n, seed)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = 1e-4
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    # secondary rays leaving instance surfaces (vertex positions of the flattened meshes)
    r = np.random.Generator(np.random.PCG64(seed + 1))
    pts = []
    for ins in sc.instances[:8]:
        m = sc.meshes[ins.mesh]
        M = ins.object_to_world.astype(np.float64)
        p = m.vertices[r.integers(0, len(m.vertices), n // 16)].astype(np.float64) @ M[:, :3].T + M[:, 3]
        pts.append(p)
    p = np.concatenate(pts)
    dd = r.normal(size=p.shape)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    sec = np.zeros((len(p), 8), np.float32)
    sec[:, 0:3] = p
    sec[:, 3] = 1e-4
    sec[:, 4:7] = dd
    sec[:, 7] = np.inf
    return np.concatenate([rays, sec])


@pytest.mark.parametrize("exact", [True, False])
def test_host_two_level_bit_exact_vs_oracle(O, exact):
    from paper_2407_19977_amd import pt
    sc = _scene(_small_meshes(), exact=exact, seed=3)
    b = pt.HostBvh(meshes=sc.meshes, instances=sc.instances)
    rays = _rays_f32(sc, 2000, 5)
    got = b.trace(rays)
    ref = O.OracleScene(sc).closest_f32(rays)
    assert ref[:, 5].sum() > 400
    assert np.array_equal(got, ref), np.argwhere((got != ref).any(1))[:5]


def test_instanced_generator_invariants():
    sc = scenes.instanced(width=64, height=36, env_size=(64, 32))
    targets = [10000, 17500, 25000, 32500, 50000]
    assert len(sc.instances) == 402
    for m, t in zip(sc.meshes[:5], targets):
        assert abs(m.n_triangles - t) <= 0.05 * t
        f = m.indices.astype(np.int64)
        e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), 1)
        _, c = np.unique(e, axis=0, return_counts=True)
        assert set(c.tolist()) == {2}  # closed
        v = m.vertices.astype(np.float64)
        n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
        assert np.einsum("ij,ij->i", v[f].mean(1), n).sum() > 0  # outward
        assert np.linalg.norm(v, axis=1).max() <= 1.3
    c = np.array([i.object_to_world[:, 3] for i in sc.instances[:400]], np.float64)
    rad = np.array([np.linalg.norm(sc.meshes[i.mesh].vertices, axis=1).max() for i in sc.instances[:400]])
    dist = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=-1) + np.eye(400) * 1e9
    assert np.all(dist > rad[:, None] + rad[None, :])  # bounding spheres never overlap: no nested media
    for i in sc.instances[:400]:
        R = i.object_to_world[:, :3].astype(np.float64)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-6) and np.linalg.det(R) > 0
    mats = sc.materials[[i.material_override for i in sc.instances[:400]]]
    glass = mats[:, 13] == 1.0        # transmission_weight
    metal = mats[:, 4] == 1.0         # base_metalness
    coat = mats[:, 17] == 1.0         # coat_weight
    assert (glass.sum(), metal.sum(), coat.sum()) == (120, 160, 120)


@pytest.mark.parametrize("n_inst", [24, 150])
def test_stack_bound_holds_and_overflow_is_an_error(n_inst):
    """The walk never needs more stack than the capacity the library gives
    the GPU lanes (3 entries per inner level plus one top-level leaf's
    instances), and a walk that runs out of stack fails the call instead of
    returning hits silently."""
    from paper_2407_19977_amd import pt
    sc = _scene(_small_meshes(), exact=False, n=n_inst, seed=4)
    b = pt.HostBvh(meshes=sc.meshes, instances=sc.instances)
    cap = b.info["stack_capacity"]
    assert cap == 3 * b.info["depth"] + b.info["max_leaf_tris"]
    rays = _rays_f32(sc, 3000, 9)
    ref = b.trace(rays)
    hits, high = b.trace_stack(rays)
    assert np.array_equal(hits, ref)
    assert 0 < high <= cap
    # every hit survives a stack exactly as deep as the deepest walk needed
    hits2, high2 = b.trace_stack(rays, capacity=high)
    assert np.array_equal(hits2, ref) and high2 == high
    with pytest.raises(pt.PtError, match="stack overflow"):
        b.trace_stack(rays, capacity=2)
    # single-level BVH: the same bound
    m = sc.meshes[2]
    b1 = pt.HostBvh(m)
    assert b1.info["stack_capacity"] == 3 * b1.info["depth"] + b1.info["max_leaf_tris"] or \
        b1.info["stack_capacity"] == 3 * b1.info["depth"] + b.info["max_leaf_tris"]
    r = np.random.Generator(np.random.PCG64(12))
    r1 = np.zeros((2000, 8), np.float32)
    r1[:, 0:3] = r.uniform(-2, 2, (2000, 3))
    d = r.uniform(-0.5, 0.5, (2000, 3)) - r1[:, 0:3]      # aimed at the mesh
    r1[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r1[:, 3] = 1e-4
    r1[:, 7] = np.inf
    h1, hw = b1.trace_stack(r1)
    assert h1[:, 5].sum() > 200 and 0 < hw <= b1.info["stack_capacity"]
    with pytest.raises(pt.PtError, match="stack overflow"):
        b1.trace_stack(r1, capacity=1)

"""CPU tests of the HIP library's host side: the C ABI loads and exports every
declared symbol, the BVH4 builder's invariants hold (Sec. 5.1.1: every child
lies inside its parent), and the traversal (compiled for the CPU) returns
bit-for-bit the closest hits of the oracle's single-precision brute force."""
import os
import re

import numpy as np
import pytest

from paper_2407_19977_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_2407_19977_amd import pt
    return pt


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(P):
    names = _declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(P.lib(), n), n
        assert n in P._SIGS, f"binding lacks {n}"
    assert "gfx950" in P.version()
    assert isinstance(P.last_error(), str)  # thread-local; earlier tests may have left a message


def _meshes():
    v, f = scenes.icosphere(3)
    ico = scenes.Mesh((v * 1.5 + 0.2).astype(np.float32), f.astype(np.int32), np.zeros(len(f), np.int32))
    r = np.random.Generator(np.random.PCG64(1))
    c = r.uniform(-1, 1, size=(2000, 1, 3))
    sv = (c + 0.1 * r.normal(size=(2000, 3, 3))).reshape(-1, 3).astype(np.float32)
    soup = scenes.Mesh(sv, np.arange(6000, dtype=np.int32).reshape(-1, 3), np.arange(2000, dtype=np.int32) % 3)
    return {"cornell": scenes.cornell().meshes[0], "icosphere": ico, "soup": soup}


def _node_fields(nodes):
    f = nodes.view(np.float32).reshape(-1, 32)
    u = nodes.view(np.uint32).reshape(-1, 32)
    lo = np.stack([f[:, 0:4], f[:, 8:12], f[:, 16:20]], -1)   # [n, 4, 3]
    hi = np.stack([f[:, 4:8], f[:, 12:16], f[:, 20:24]], -1)
    return lo, hi, u[:, 24:28], u[:, 28]


@pytest.mark.parametrize("name", ["cornell", "icosphere", "soup"])
def test_bvh4_invariants(P, name):
    mesh = _meshes()[name]
    b = P.HostBvh(mesh)
    nodes, tris = b.arrays()
    n_tri = mesh.indices.shape[0]
    assert b.info["n_tris"] == n_tri and nodes.shape[1] == 128 and tris.shape[1] == 48
    tf = tris.view(np.float32).reshape(-1, 12)
    tu = tris.view(np.uint32).reshape(-1, 12)
    prim = tu[:, 3]
    assert np.array_equal(np.sort(prim), np.arange(n_tri))          # each triangle exactly once
    # triangle records carry the input vertices and material ids
    V = mesh.vertices[mesh.indices[prim]]
    assert np.array_equal(tf[:, [0, 1, 2]], V[:, 0]) and np.array_equal(tf[:, [4, 5, 6]], V[:, 1])
    assert np.array_equal(tf[:, [8, 9, 10]], V[:, 2]) and np.array_equal(tu[:, 7], mesh.material_ids[prim])
    lo, hi, child, nvalid = _node_fields(nodes)
    covered = np.zeros(n_tri, np.int64)
    seen_nodes = {0}
    depth_max = 0
    stack = [(0, 1)]
    while stack:
        ni, d = stack.pop()
        depth_max = max(depth_max, d)
        for c in range(4):
            ref = int(child[ni, c])
            if ref == 0xFFFFFFFF:
                continue
            if ref & 0x80000000:
                cnt = (ref >> 27) & 7
                first = ref & ((1 << 27) - 1)
                assert 1 <= cnt <= 4
                covered[first:first + cnt] += 1
                pts = tf[first:first + cnt][:, [0, 1, 2, 4, 5, 6, 8, 9, 10]].reshape(-1, 3)
                assert np.all(pts >= lo[ni, c]) and np.all(pts <= hi[ni, c])
                depth_max = max(depth_max, d + 1)
            else:
                assert ref not in seen_nodes
                seen_nodes.add(ref)
                # a child node's boxes lie inside the parent's box for it
                valid = child[ref] != 0xFFFFFFFF
                assert np.all(lo[ref][valid] >= lo[ni, c]) and np.all(hi[ref][valid] <= hi[ni, c])
                stack.append((ref, d + 1))
    assert np.all(covered == 1)
    assert len(seen_nodes) == nodes.shape[0]
    assert depth_max == b.info["depth"]
    assert b.info["max_leaf_tris"] <= 4


def _rays(mesh, n, seed):
    """Primary-like, secondary (from triangle points) and grazing rays."""
    r = np.random.Generator(np.random.PCG64(seed))
    v = mesh.vertices.astype(np.float64)
    lo, hi = v.min(0), v.max(0)
    ext = hi - lo
    o1 = r.uniform(lo - 0.5 * ext, hi + 0.5 * ext, size=(n, 3))
    d1 = r.normal(size=(n, 3))
    tri = v[mesh.indices[r.integers(0, len(mesh.indices), n)]]
    w = r.dirichlet([1, 1, 1], size=n)
    o2 = np.einsum("nk,nkj->nj", w, tri)
    d2 = r.normal(size=(n, 3))
    # grazing: along a triangle edge direction, starting near the triangle
    e = tri[:, 1] - tri[:, 0]
    o3 = tri[:, 0] - 0.3 * e + 1e-4 * r.normal(size=(n, 3))
    d3 = e + 1e-3 * r.normal(size=(n, 3))
    o = np.concatenate([o1, o2, o3])
    d = np.concatenate([d1, d2, d3])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((len(o), 8), np.float32)
    rays[:, 0:3] = o
    rays[:, 3] = 1e-5 * np.linalg.norm(ext)
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


@pytest.mark.parametrize("name", ["cornell", "icosphere", "soup"])
def test_host_traversal_bit_exact_vs_oracle_brute_force(P, O, name):
    mesh = _meshes()[name]
    b = P.HostBvh(mesh)
    rays = _rays(mesh, 1500, 7)
    got = b.trace(rays)
    cam = scenes.Camera((0, 0, -3), (0, 0, 0), (0, 1, 0), 40.0, 8, 8)
    sc = scenes.Scene("t", [mesh], [], np.stack([scenes.lambert((0.5, 0.5, 0.5))] * 8), None, cam, 1, 1)
    ref = O.OracleScene(sc).closest_f32(rays)
    assert ref[:, 5].sum() > 300
    assert np.array_equal(got, ref), np.argwhere((got != ref).any(1))[:5]

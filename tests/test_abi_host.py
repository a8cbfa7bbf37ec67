"""C ABI checks that need no GPU: the library loads and exports every call
declared in include/neuvv.h; the host-side octree build is checked against an
independent construction; argument errors come back as status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2202_06088_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2202_06088_amd.build import build_library
        build_library()
    return _lib.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "neuvv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(neuvv_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert lib.neuvv_version() >= 100


def reference_tree(depth, ijk):
    """Independent construction: dict from (level, prefix) to node, breadth first,
    siblings ordered by the interleaved prefix bits."""
    def prefix(c, lvl):
        sh = depth - lvl
        return tuple(int(v) >> sh for v in c)

    def key(p, lvl):
        k = 0
        for b in range(lvl - 1, -1, -1):
            for a in (2, 1, 0):
                k = (k << 1) | ((p[a] >> b) & 1)
        return k

    levels = [[()]]
    for lvl in range(1, depth):
        ps = sorted({prefix(c, lvl) for c in ijk}, key=lambda p: key(p, lvl))
        levels.append(ps)
    index = {}
    n = 0
    for lvl, ps in enumerate(levels):
        for p in ps:
            index[(lvl, p)] = n
            n += 1
    leaves = sorted(range(len(ijk)), key=lambda q: key(tuple(int(v) for v in ijk[q]), depth))
    slot = {q: s for s, q in enumerate(leaves)}
    child = -np.ones((n, 8), np.int32)
    for lvl in range(1, depth):
        for p in levels[lvl]:
            parent = index[(lvl - 1, tuple(v >> 1 for v in p) if lvl > 1 else ())]
            o = (p[0] & 1) | ((p[1] & 1) << 1) | ((p[2] & 1) << 2)
            child[parent, o] = index[(lvl, p)]
    for q, c in enumerate(ijk):
        c = tuple(int(v) for v in c)
        parent = index[(depth - 1, prefix(c, depth - 1) if depth > 1 else ())]
        o = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2)
        child[parent, o] = slot[q]
    return child, np.array([slot[q] for q in range(len(ijk))], np.int64)


@pytest.mark.parametrize("depth,n,seed", [(1, 3, 0), (2, 20, 1), (3, 100, 2), (5, 700, 3), (12, 50, 4)])
def test_build_matches_reference(lib, depth, n, seed):
    from paper_2202_06088_amd.voctree import build_child_table
    rng = np.random.default_rng(seed)
    G = 1 << depth
    flat = rng.choice(G ** 3, size=min(n, G ** 3), replace=False)
    ijk = np.stack([flat % G, (flat // G) % G, flat // (G * G)], -1).astype(np.int32)
    child, slots, box = build_child_table(depth, ijk, with_box=True)
    ref_child, ref_slots = reference_tree(depth, ijk)
    assert np.array_equal(child, ref_child)
    assert np.array_equal(slots, ref_slots)
    assert np.array_equal(box[:3], ijk.min(0)) and np.array_equal(box[3:], ijk.max(0) + 1)


def test_build_empty_and_errors(lib):
    from paper_2202_06088_amd.voctree import build_child_table
    child, slots, box = build_child_table(4, np.zeros((0, 3), np.int32), with_box=True)
    assert child.shape == (1, 8) and np.all(child == -1) and slots.shape == (0,)
    assert np.all(box == 0)
    ijk = np.array([[0, 0, 0], [1, 2, 3], [0, 0, 0]], np.int32)
    with pytest.raises(_lib.NeuvvError) as e:
        _lib.neuvv_build_voctree(3, ijk)
    assert e.value.code == -3
    with pytest.raises(_lib.NeuvvError) as e:
        _lib.neuvv_build_voctree(2, np.array([[0, 4, 0]], np.int32))
    assert e.value.code == -2
    with pytest.raises(_lib.NeuvvError) as e:
        _lib.neuvv_build_voctree(13, np.array([[0, 0, 0]], np.int32))
    assert e.value.code == -2
    ijk = np.array([[0, 0, 0], [3, 3, 3]], np.int32)
    n = _lib.neuvv_build_voctree(2, ijk)
    small = np.empty((n - 1, 8), np.int32)
    with pytest.raises(_lib.NeuvvError) as e:
        _lib.neuvv_build_voctree(2, ijk, small, n - 1)
    assert e.value.code == -4
    assert "capacity" in _lib.neuvv_last_error()


def test_argument_errors_without_launch(lib):
    # failures detected on the host before anything touches a device
    assert lib.neuvv_render(None, None, 1, None, None, None, 0.0, 0, 0.0, None, None, None, None, None) == -1
    t = _lib.neuvv_tree()
    t.depth, t.K, t.C, t.dtype, t.n_nodes, t.n_leaves, t.T = 9, 14, 8, 0, 1, 0, 1
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    t.K, t.depth = 16, 13
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -2
    t.K, t.depth, t.child, t.basis, t.gamma = 16, 3, 8, 8, 8    # non-NULL placeholders, never dereferenced
    for bad in ((0, 0, 0, 9, 1, 1), (2, 0, 0, 2, 1, 1), (-1, 0, 0, 1, 1, 1)):
        for i in range(6):
            t.box[i] = bad[i]
        assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                                None) == -2
    t.layout = 3
    for i in range(6):
        t.box[i] = 0
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    t.layout = 0
    t.depth, t.dtype = 9, 7
    assert lib.neuvv_render_backward(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None,
                                     None, None, None, None, None, None) == -1
    assert lib.neuvv_compose(0, 10, None, None, None, None, None, None, None) == -2
    assert lib.neuvv_compose(17, 10, None, None, None, None, None, None, None) == -2
    assert lib.neuvv_compose(2, 10, None, None, None, None, None, None, None) == -1
    assert lib.neuvv_eval_hh(31, 1, None, None, None, None) == -2
    cam = _lib.make_camera(0, 10, 1.0, 1.0, 0.0, 0.0, np.zeros(12))
    assert lib.neuvv_pinhole_rays(ctypes.byref(cam), 0, None, None, None, None) == -2
    assert lib.neuvv_pack_leaves(16, 8, 5, 0, 1, None, None, None, None, None, None) == -5
    assert lib.neuvv_pack_leaves(16, 8, 0, 7, 1, None, None, None, None, None, None) == -5
    a, b = _lib.neuvv_payload_words(16, 8, _lib.F32, 10)
    assert (a, b) == (12 * 10 * 4, 2 * 10 * 4)
    a, b = _lib.neuvv_payload_words(16, 8, _lib.F16, 10)
    assert (a, b) == (6 * 10 * 8, 1 * 10 * 8)
    a, b = _lib.neuvv_payload_words(14, 31, _lib.F32, 3)
    assert (a, b) == (11 * 3 * 4, 8 * 3 * 4)

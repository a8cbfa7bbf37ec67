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
    return sorted(set(re.findall(r"^\s*(?:int64_t|int32_t|int|const char\*)\s+(neuvv_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert lib.neuvv_version() >= 200


def reference_tree(depth, ijk):
    """Independent construction of the node table from its definition: node
    levels w = 0..ceil(D/2)-1 with b_0 = 1 for odd D (else 2) and b_w = 2 after,
    node edge e_w (e_0 = D, e_(w+1) = e_w - b_w); nodes are the distinct cubes
    (coordinates >> e_w) holding a leaf, breadth first, Morton order within a
    level; a node's mask bit q = Morton code of the child's local coordinates."""
    L = (depth + 1) // 2
    b = [1 if (w == 0 and depth % 2) else 2 for w in range(L)]
    e = [depth]
    for w in range(L):
        e.append(e[-1] - b[w])

    def morton(p, nbits):
        k = 0
        for bit in range(nbits - 1, -1, -1):
            for a in (2, 1, 0):
                k = (k << 1) | ((p[a] >> bit) & 1)
        return k

    cells = [tuple(int(v) for v in c) for c in ijk]
    levels = []
    for w in range(L):
        ps = sorted({tuple(v >> e[w] for v in c) for c in cells}, key=lambda p: morton(p, depth))
        levels.append(ps if ps else [(0, 0, 0)])
    index = {}
    n = 0
    for w, ps in enumerate(levels):
        for p in ps:
            index[(w, p)] = n
            n += 1
    order = sorted(range(len(cells)), key=lambda q: morton(cells[q], depth))
    slot = {q: s for s, q in enumerate(order)}
    kids = {r: [] for r in range(n)}          # node row -> [(bit q, child index)]
    for w in range(1, L):
        for p in levels[w]:
            parent = tuple(v >> b[w - 1] for v in p)
            local = tuple(v - (u << b[w - 1]) for v, u in zip(p, parent))
            kids[index[(w - 1, parent)]].append((morton(local, b[w - 1]), index[(w, p)]))
    for q, c in enumerate(cells):
        parent = tuple(v >> b[L - 1] for v in c)
        local = tuple(v - (u << b[L - 1]) for v, u in zip(c, parent))
        kids[index[(L - 1, parent)]].append((morton(local, b[L - 1]), slot[q]))
    nodes = np.zeros((n, 4), np.int32)
    for r, lst in kids.items():
        if not lst:
            continue
        lst.sort()
        mask = 0
        for q, _ in lst:
            mask |= 1 << q
        nodes[r, 0] = np.uint32(mask & 0xffffffff).view(np.int32)
        nodes[r, 1] = np.uint32(mask >> 32).view(np.int32)
        nodes[r, 2] = lst[0][1]
        # occupied children are consecutive in bit order
        assert [c for _, c in lst] == list(range(lst[0][1], lst[0][1] + len(lst)))
    return nodes, np.array([slot[q] for q in range(len(cells))], np.int64)


def expand_leaves(depth, nodes):
    """Leaf cells reached from the root by following every set mask bit."""
    L = (depth + 1) // 2
    b = [1 if (w == 0 and depth % 2) else 2 for w in range(L)]
    out = {}

    def rec(row, w, origin):
        m = (int(np.uint32(nodes[row, 0])) | (int(np.uint32(nodes[row, 1])) << 32))
        rank = 0
        for q in range(64):
            if not (m >> q) & 1:
                continue
            local = [0, 0, 0]
            for bit in range(b[w]):
                for a in range(3):
                    local[a] |= ((q >> (3 * bit + a)) & 1) << bit
            cell = tuple((o << b[w]) + l for o, l in zip(origin, local))
            idx = int(nodes[row, 2]) + rank
            rank += 1
            if w == L - 1:
                out[cell] = idx
            else:
                rec(idx, w + 1, cell)

    rec(0, 0, (0, 0, 0))
    return out


@pytest.mark.parametrize("depth,n,seed", [(1, 3, 0), (2, 20, 1), (3, 100, 2), (4, 300, 5), (5, 700, 3),
                                          (6, 2000, 6), (12, 50, 4)])
def test_build_matches_reference(lib, depth, n, seed):
    from paper_2202_06088_amd.voctree import build_node_table
    rng = np.random.default_rng(seed)
    G = 1 << depth
    flat = rng.choice(G ** 3, size=min(n, G ** 3), replace=False)
    ijk = np.stack([flat % G, (flat // G) % G, flat // (G * G)], -1).astype(np.int32)
    nodes, slots, box = build_node_table(depth, ijk, with_box=True)
    ref_nodes, ref_slots = reference_tree(depth, ijk)
    assert np.array_equal(nodes, ref_nodes)
    assert np.array_equal(slots, ref_slots)
    assert np.array_equal(box[:3], ijk.min(0)) and np.array_equal(box[3:], ijk.max(0) + 1)
    # the table reaches exactly the input cells, each at its slot
    reached = expand_leaves(depth, nodes)
    assert reached == {tuple(int(v) for v in c): int(s) for c, s in zip(ijk, slots)}


def test_build_empty_and_errors(lib):
    from paper_2202_06088_amd.voctree import build_node_table
    nodes, slots, box = build_node_table(4, np.zeros((0, 3), np.int32), with_box=True)
    assert nodes.shape == (1, 4) and np.all(nodes == 0) and slots.shape == (0,)
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
    ijk = np.array([[0, 0, 0], [3, 3, 3], [7, 0, 5]], np.int32)
    n = _lib.neuvv_build_voctree(3, ijk)
    small = np.empty((n - 1, 4), np.int32)
    with pytest.raises(_lib.NeuvvError) as e:
        _lib.neuvv_build_voctree(3, ijk, small, n - 1)
    assert e.value.code == -4
    assert "capacity" in _lib.neuvv_last_error()


def test_argument_errors_without_launch(lib):
    # failures detected on the host before anything touches a device
    assert lib.neuvv_render(None, None, 1, None, None, None, 0.0, 0, 0.0, None, None, None, None, None) == -1
    t = _lib.neuvv_tree()
    t.depth, t.K, t.C, t.dtype, t.n_nodes, t.n_leaves, t.T = 9, 15, 8, 0, 1, 0, 1
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    t.K, t.C = 16, 12
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    # the compiled shapes of the global-hyperangle form (K in {14, 16, 30}, C in {8, 31}): a call
    # with no rays passes the checks and launches nothing
    t.nodes, t.basis, t.gamma = 16, 8, 8             # non-NULL placeholders, never dereferenced
    t.K, t.C = 16, 8
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1                 # the walk needs the brick directory
    assert "dir" in _lib.neuvv_last_error()
    t.dir = 6                                        # directory entries are 4-byte aligned
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    assert "aligned" in _lib.neuvv_last_error()
    t.dir = 16
    for K in (14, 16, 30):
        for C in (8, 31):
            t.K, t.C = K, C
            assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None,
                                    None, None) == 0, (K, C, _lib.neuvv_last_error())
    t.density = 2                                    # no such activation
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    t.density = 0
    t.nodes, t.basis, t.gamma = None, None, None
    t.K, t.depth = 16, 13
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -2
    t.K, t.depth, t.nodes, t.basis, t.gamma = 16, 3, 16, 8, 8    # non-NULL placeholders, never dereferenced
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
    t.nodes = 8                                     # node rows must be 16-byte aligned
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    assert "aligned" in _lib.neuvv_last_error()
    t.nodes = 16
    t.depth, t.dtype = 9, 7
    assert lib.neuvv_render_backward(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None,
                                     None, None, None, None, None, None, None) == -1
    # per-point hyperangle form: only K = 14, C = 31, Cg = 31 is compiled, and it needs its basis
    t.depth, t.dtype = 9, 0
    t.K, t.C, t.Cg = 16, 8, 31
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    t.K, t.C, t.Cg, t.gamma = 14, 31, 31, None
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    assert "basis_g" in _lib.neuvv_last_error()
    t.basis_g = 8
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == 0
    t.Cg = 0                                        # the global form of K = 14, C = 31 needs its gamma table
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    assert "gamma" in _lib.neuvv_last_error()
    t.K, t.C, t.Cg, t.edit, t.gamma = 30, 8, 0, 64, 8  # edits are compiled for K = 16, C = 8 only
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    t.gamma = None
    # appearance edits: K=16 C=8 form only, 16-byte aligned rows; terminal-leaf and paint arguments
    t.K, t.C, t.Cg, t.edit = 14, 31, 31, 64
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -5
    t.K, t.C, t.Cg, t.gamma, t.edit = 16, 8, 0, 8, 72
    assert lib.neuvv_render(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None,
                            None) == -1
    t.edit = None
    assert lib.neuvv_find_terminal_leaves(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 1.0, None,
                                          None) == -2
    assert lib.neuvv_find_terminal_leaves(ctypes.byref(t), None, 0, None, None, None, 0.0, 0, 0.99, None,
                                          None) == 0
    # traced calls: the trace buffer's size, alignment and room; both forms
    assert _lib.neuvv_trace_bytes(10, 5) == 2048 + 256 + 5 * 32
    assert lib.neuvv_trace_bytes(-1, 5) == -1
    args = (None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None)
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, None, 16, None) == -1
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, 8, 16, None) == -1
    assert "aligned" in _lib.neuvv_last_error()
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, 256, -1, None) == -2
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, 256, 2 ** 31, None) == -2
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, 256, 16, None) == 0
    bargs = (None, 0, None, None, None, 0.0, 0, 0.0, None, None, None, None, None, None, None, None)
    assert lib.neuvv_render_backward_trace(ctypes.byref(t), *bargs, None, 16, None) == -1
    assert lib.neuvv_render_backward_trace(ctypes.byref(t), *bargs, 256, -3, None) == -2
    assert lib.neuvv_render_backward_trace(ctypes.byref(t), *bargs, 256, 16, None) == 0
    t.K, t.C, t.Cg, t.basis_g = 14, 31, 31, 8
    assert lib.neuvv_render_trace(ctypes.byref(t), *args, 256, 16, None) == 0
    assert lib.neuvv_render_backward_trace(ctypes.byref(t), *bargs, 256, 16, None) == 0
    assert lib.neuvv_render_backward_trace(ctypes.byref(t), *bargs, 256, -1, None) == -2
    t.K, t.C, t.Cg, t.basis_g = 16, 8, 0, None
    assert lib.neuvv_paint(3, None, None, 1.0, 0.0, 10, None, None) == -1
    assert lib.neuvv_paint(-1, None, None, 1.0, 0.0, 10, None, None) == -2
    assert lib.neuvv_paint(0, None, None, 1.0, 0.0, 10, None, None) == 0
    assert lib.neuvv_compose(0, 10, None, None, None, None, None, None, None) == -2
    assert lib.neuvv_compose(17, 10, None, None, None, None, None, None, None) == -2
    assert lib.neuvv_compose(2, 10, None, None, None, None, None, None, None) == -1
    assert lib.neuvv_eval_hh(31, 1, None, None, None, None) == -2
    cam = _lib.make_camera(0, 10, 1.0, 1.0, 0.0, 0.0, np.zeros(12))
    assert lib.neuvv_pinhole_rays(ctypes.byref(cam), 0, None, None, None, None) == -2
    assert lib.neuvv_pack_leaves(16, 8, 5, 0, 1, None, None, None, None, None, None) == -5
    assert lib.neuvv_pack_leaves(16, 8, 0, 7, 1, None, None, None, None, None, None) == -5
    assert lib.neuvv_pack_rows(0, 0, 0, 1, None, None, None, None) == -2
    assert lib.neuvv_pack_rows(31, 5, 0, 1, None, None, None, None) == -5
    assert lib.neuvv_pack_rows(31, 0, 1, 1, None, None, None, None) == -1
    assert lib.neuvv_pack_rows(31, 0, 1, 0, None, None, None, None) == 0
    assert _lib.neuvv_grad_row_elems(16, 8) == 64
    assert _lib.neuvv_grad_row_elems(14, 31, 31) == 128
    # lighting calls: sizes, sigma, in-place, light parameters
    assert lib.neuvv_blur(0, 4, 8, 1.0, 16, None) == -2
    assert lib.neuvv_blur(4, 4, 8, 0.0, 16, None) == -2
    assert lib.neuvv_blur(4, 4, 8, 17.0, 16, None) == -2
    assert lib.neuvv_blur(4, 4, 8, 1.0, 8, None) == -1
    assert lib.neuvv_blur(4, 4, None, 1.0, 16, None) == -1
    cam = _lib.make_camera(8, 8, 4.0, 4.0, 4.0, 4.0, np.eye(3, 4, dtype=np.float32))
    light = _lib.make_light(cam, 0.0, (1, 1, 1), (0, 0, 0), 1.5, 0.0)
    assert lib.neuvv_shade(ctypes.byref(light), None, 0, None, None, None, None, None, None, None) == -2
    light = _lib.make_light(cam, 0.0, (1, 1, 1), (0, 0, 0), 0.5, -1.0)
    assert lib.neuvv_shade(ctypes.byref(light), None, 0, None, None, None, None, None, None, None) == -2
    light = _lib.make_light(cam, 0.0, (1, 1, 1), (0, 0, 0), 0.5, 2.0)
    assert lib.neuvv_shade(ctypes.byref(light), None, 5, None, None, None, None, None, None, None) == -1
    assert lib.neuvv_shade(ctypes.byref(light), None, 0, None, None, None, None, None, None, None) == 0
    assert lib.neuvv_shade(None, None, 0, None, None, None, None, None, None, None) == -1
    assert lib.neuvv_grad_row_elems(14, 31, 65) == -2
    a, b = _lib.neuvv_payload_words(16, 8, _lib.F32, 10)
    assert (a, b) == (12 * 10 * 4, 2 * 10 * 4)
    a, b = _lib.neuvv_payload_words(16, 8, _lib.F16, 10)
    assert (a, b) == (6 * 10 * 8, 1 * 10 * 8)
    a, b = _lib.neuvv_payload_words(14, 31, _lib.F32, 3)
    assert (a, b) == (11 * 3 * 4, 8 * 3 * 4)


def test_directory_sizes_and_argument_errors(lib):
    """Brick directory: E^3 entries with E = 2^(D-2) (1 for D <= 2); arguments checked before any
    launch."""
    assert [_lib.neuvv_directory_entries(d) for d in (1, 2, 3, 9, 10, 12)] == [1, 1, 8, 128 ** 3, 256 ** 3,
                                                                              1024 ** 3]
    for d in (0, 13):
        assert lib.neuvv_directory_entries(d) == -1
    assert lib.neuvv_build_directory(9, 1, 16, 16, 128 ** 3 - 1, None) == -4
    assert "needs" in _lib.neuvv_last_error()
    assert lib.neuvv_build_directory(13, 1, 16, 16, 1 << 40, None) == -2
    assert lib.neuvv_build_directory(9, 0, 16, 16, 128 ** 3, None) == -2
    assert lib.neuvv_build_directory(9, 1, None, 16, 128 ** 3, None) == -1
    assert lib.neuvv_build_directory(9, 1, 8, 16, 128 ** 3, None) == -1
    assert lib.neuvv_build_directory(9, 1, 16, 6, 128 ** 3, None) == -1

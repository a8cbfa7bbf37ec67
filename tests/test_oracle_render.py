"""Pins for the FP64 oracle renderer (Sec. 4.3 "Rendering", Eq. 4, 5, 8, 9, 13).

The oracle is checked against: a brute-force plane-crossing renderer that
writes Eq. 8 literally (tiny trees, tests/bruteforce.py), the closed form of
a single voxel, the telescoping identity sum(w) + T_final = 1, the merge of two
equal-colour voxels into one of summed optical depth, the miss case, integer
times selecting basis rows, central finite differences for the gradient, and
the geometric invariances of the instance transform (Eq. 13).
"""
import math

import numpy as np
import pytest

import bruteforce as BF
from oracle.hh import hh_basis
from workloads import make_scene, random_rays, special_rays, random_rotation


def tiny_scene(depth=3, n_leaves=None, seed=0, K=16, C=8, T=6):
    rng = np.random.default_rng(seed)
    G = 1 << depth
    allc = np.stack(np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij"), -1).reshape(-1, 3)
    n = n_leaves or (G ** 3) // 3
    ijk = allc[rng.choice(allc.shape[0], n, replace=False)].astype(np.int32)
    hh = rng.normal(0, 0.5, (n, 3, K)).astype(np.float32)
    wsig = rng.normal(0, 1, (n, C)).astype(np.float32)
    basis = rng.normal(0, 1, (T, C)).astype(np.float32)
    gamma = (math.pi * (np.arange(T) + 0.5) / T).astype(np.float32)
    return ijk, hh, wsig, basis, gamma


@pytest.mark.parametrize("depth,t_stop,seed", [(2, 0.0, 0), (3, 0.0, 1), (3, 0.05, 2), (4, 1e-3, 3)])
def test_oracle_matches_bruteforce(oracle_lib, depth, t_stop, seed):
    ijk, hh, wsig, basis, gamma = tiny_scene(depth, seed=seed)
    G = 1 << depth
    rng = np.random.default_rng(seed + 100)
    o1, d1 = random_rays(G, 40, rng, inside_frac=0.25)
    o2, d2 = special_rays(G)
    o = np.concatenate([o1, o2])
    d = np.concatenate([d1, d2])
    t = 2.0
    res = oracle_lib.render(depth, ijk, hh, wsig, basis, gamma, o, d, None, t, t_stop)
    for r in range(o.shape[0]):
        C, A, D, ns = BF.render(depth, ijk, hh, wsig, basis, gamma, o[r].astype(np.float64),
                                d[r].astype(np.float64), t, t_stop)
        assert np.allclose(res["rgb"][r], C, rtol=0, atol=1e-12), r
        assert abs(res["alpha"][r] - A) < 1e-12, r
        assert (math.isinf(D) and math.isinf(res["depth"][r])) or abs(res["depth"][r] - D) < 1e-9, r
        assert res["nsamp"][r] == ns, (r, res["nsamp"][r], ns)


def test_single_voxel_closed_form(oracle_lib):
    # one leaf at (1,2,3) in a depth-3 grid; K=1 so c = sigmoid(w / (pi sqrt 2))
    ijk = np.array([[1, 2, 3]], np.int32)
    hh = np.array([[[0.7], [-0.4], [1.3]]], np.float32)
    wsig = np.array([[0.9, -0.3]], np.float32)
    basis = np.array([[1.0, 2.0], [0.5, -1.0]], np.float32)
    gamma = np.array([0.4, 1.1], np.float32)
    x = float(wsig[0, 0]) * 1.0 + float(wsig[0, 1]) * 2.0
    sig = math.log1p(math.exp(x))
    h0 = 1.0 / (math.pi * math.sqrt(2.0))
    c = np.array([1 / (1 + math.exp(-float(v) * h0)) for v in hh[0, :, 0]])
    cases = [  # (origin, direction, segment length, midpoint distance)
        ((1.5, 2.5, -4.0), (0, 0, 1), 1.0, 7.5),
        ((1.25, -10.0, 3.75), (0, 2, 0), 1.0, 12.5),
        ((0.0, 1.0, 2.0), (1, 1, 1), math.sqrt(3.0), 1.5 * math.sqrt(3.0)),
    ]
    for o, d, ell, mid in cases:
        res = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, np.array([o]), np.array([d]), None, 0.0, 0.0)
        a = 1 - math.exp(-sig * ell)
        assert abs(res["alpha"][0] - a) < 1e-14
        assert np.abs(res["rgb"][0] - a * c).max() < 1e-14
        assert abs(res["depth"][0] - mid) < 1e-12
        assert res["nsamp"][0] == 1


def test_weights_plus_transmittance_is_one(oracle_lib):
    sc = make_scene(5, 3000, "random", seed=7, T=10)
    rng = np.random.default_rng(8)
    o, d = random_rays(sc.G, 400, rng)
    for t_stop in (0.0, 1e-4, 0.1):
        res = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 3.0, t_stop)
        assert np.abs(res["alpha"] + res["tfinal"] - 1.0).max() < 1e-12
        if t_stop > 0:
            stopped = res["tfinal"] < t_stop
            assert stopped.any()


def test_equal_colour_voxels_merge(oracle_lib):
    # two adjacent leaves along x with identical colour coefficients: the pair renders as one
    # voxel of optical depth sigma1 * l1 + sigma2 * l2
    ijk = np.array([[3, 4, 4], [4, 4, 4]], np.int32)
    hh = np.zeros((2, 3, 16), np.float32)
    hh[:, :, 0] = [0.3, -0.8, 1.1]
    hh[:, :, 5] = [0.2, 0.1, -0.4]
    wsig = np.array([[0.5, 1.0], [-1.0, 0.25]], np.float32)
    basis = np.array([[1.0, 1.0]], np.float32)
    gamma = np.array([1.0], np.float32)
    o = np.array([[0.0, 4.3, 4.6]], np.float32)
    d = np.array([[1.0, 0.05, -0.02]], np.float32)
    res = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 0.0, 0.0)
    dd = d[0].astype(np.float64)
    n = np.linalg.norm(dd)
    l1 = (4 - 3) / dd[0] * n
    l2 = (5 - 4) / dd[0] * n
    s1 = math.log1p(math.exp(1.5))
    s2 = math.log1p(math.exp(-0.75))
    h = hh_basis(16, dd / n, 1.0)
    c = 1 / (1 + np.exp(-(hh[0].astype(np.float64) @ h)))
    a = 1 - math.exp(-(s1 * l1 + s2 * l2))
    assert abs(res["alpha"][0] - a) < 1e-13
    assert np.abs(res["rgb"][0] - a * c).max() < 1e-13


def test_miss_and_zero_direction(oracle_lib):
    ijk, hh, wsig, basis, gamma = tiny_scene(3)
    o = np.array([[-1, 4, 4], [4, 4, 4], [20, 20, 20]], np.float32)
    d = np.array([[0, 1, 0], [0, 0, 0], [1, 1, 1]], np.float32)
    res = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 0.0, 0.0)
    assert np.all(res["rgb"] == 0) and np.all(res["alpha"] == 0)
    assert np.all(np.isinf(res["depth"])) and np.all(res["nsamp"] == 0)


def test_softplus_zero_and_integer_time(oracle_lib):
    ijk = np.array([[0, 0, 0]], np.int32)
    hh = np.zeros((1, 3, 16), np.float32)
    wsig = np.array([[1.0, 0.0]], np.float32)
    basis = np.array([[0.0, 5.0], [2.0, 5.0], [-1.0, 5.0]], np.float32)
    gamma = np.array([0.1, 0.2, 0.3], np.float32)
    o = np.array([[0.5, 0.5, -1.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    for t, x in ((0.0, 0.0), (1.0, 2.0), (2.0, -1.0), (0.5, 1.0), (1.25, 2.0 - 0.75), (7.0, -1.0), (-3.0, 0.0)):
        res = oracle_lib.render(1, ijk, hh, wsig, basis, gamma, o, d, None, t, 0.0)
        sig = math.log(2.0) if x == 0.0 else math.log1p(math.exp(x))
        assert abs(res["alpha"][0] - (1 - math.exp(-sig))) < 1e-14, t
        assert np.abs(res["rgb"][0] - 0.5 * res["alpha"][0]).max() < 1e-15   # zero hh -> c = 1/2


def test_wrapped_time_offset(oracle_lib):
    from oracle.core import Instance
    ijk = np.array([[0, 0, 0]], np.int32)
    hh = np.zeros((1, 3, 16), np.float32)
    wsig = np.array([[1.0]], np.float32)
    basis = np.array([[0.0], [1.0], [2.0], [3.0]], np.float32)
    gamma = np.array([0.1, 0.2, 0.3, 0.4], np.float32)
    o = np.array([[0.5, 0.5, -1.0]], np.float32)
    d = np.array([[0.0, 0.0, 1.0]], np.float32)
    # T = 4: the last frame is held on [3, 4); wrapping is modulo 4, clamping is into [0, 3]
    for t, off, wrap, x in ((1.0, 2.5, True, 3.0), (1.0, 2.5, False, 3.0), (3.5, 0.0, True, 3.0),
                            (0.0, -0.5, True, 3.0), (0.0, -1.5, True, 2.5), (9.0, -1.0, True, 0.0),
                            (5.25, 0.0, True, 1.25), (1.0, -2.0, False, 0.0), (0.5, 0.25, False, 0.75)):
        inst = Instance(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, off, wrap)
        res = oracle_lib.render(1, ijk, hh, wsig, basis, gamma, o, d, None, t, 0.0, inst=inst)
        assert abs(res["alpha"][0] - (1 - math.exp(-math.log1p(math.exp(x))))) < 1e-14, (t, off, wrap)


def _loss_and_grads(oracle_lib, depth, ijk, hh, wsig, basis, gamma, o, d, t, gC, gA, inst=None):
    res = oracle_lib.render(depth, ijk, hh, wsig, basis, gamma, o, d, t, 0.0, 0.0, inst=inst, g_rgb=gC, g_alpha=gA)
    return float((res["rgb"] * gC).sum() + (res["alpha"] * gA).sum()), res


def test_gradient_matches_finite_differences(oracle_lib):
    ijk, hh, wsig, basis, gamma = tiny_scene(3, n_leaves=60, seed=11, T=5)
    hh = hh.astype(np.float64)
    wsig = wsig.astype(np.float64)
    basis = basis.astype(np.float64)
    rng = np.random.default_rng(12)
    o, d = random_rays(8, 30, rng)
    t = rng.uniform(0, 4, 30).astype(np.float32)
    gC = rng.normal(size=(30, 3))
    gA = rng.normal(size=30)
    L0, res = _loss_and_grads(oracle_lib, 3, ijk, hh, wsig, basis, gamma, o, d, t, gC, gA)
    eps = 1e-6

    def fd(arr, idx):
        a = arr.copy(); a[idx] += eps
        b = arr.copy(); b[idx] -= eps
        return a, b

    touched = np.unique(np.nonzero(np.abs(res["grad_wsig"]).sum(1))[0])
    assert touched.size > 5
    for q in touched[:8]:
        for idx in ((q, 0, 0), (q, 1, 3), (q, 2, 15), (q, 0, 7)):
            a, b = fd(hh, idx)
            La = _loss_and_grads(oracle_lib, 3, ijk, a, wsig, basis, gamma, o, d, t, gC, gA)[0]
            Lb = _loss_and_grads(oracle_lib, 3, ijk, b, wsig, basis, gamma, o, d, t, gC, gA)[0]
            assert abs((La - Lb) / (2 * eps) - res["grad_hh"][idx]) < 1e-7 * max(1, abs(res["grad_hh"][idx]))
        for c in range(wsig.shape[1]):
            a, b = fd(wsig, (q, c))
            La = _loss_and_grads(oracle_lib, 3, ijk, hh, a, basis, gamma, o, d, t, gC, gA)[0]
            Lb = _loss_and_grads(oracle_lib, 3, ijk, hh, b, basis, gamma, o, d, t, gC, gA)[0]
            assert abs((La - Lb) / (2 * eps) - res["grad_wsig"][q, c]) < 1e-7 * max(1, abs(res["grad_wsig"][q, c]))
    for i in range(basis.shape[0]):
        for c in (0, 5):
            a, b = fd(basis, (i, c))
            La = _loss_and_grads(oracle_lib, 3, ijk, hh, wsig, a, gamma, o, d, t, gC, gA)[0]
            Lb = _loss_and_grads(oracle_lib, 3, ijk, hh, wsig, b, gamma, o, d, t, gC, gA)[0]
            assert abs((La - Lb) / (2 * eps) - res["grad_basis"][i, c]) < 1e-7 * max(1, abs(res["grad_basis"][i, c]))


def test_identity_instance_equals_plain(oracle_lib):
    from oracle.core import Instance
    sc = make_scene(5, 3000, "random", seed=3, T=10)
    o, d = random_rays(sc.G, 200, np.random.default_rng(4))
    a = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 2.5, 1e-4)
    inst = Instance(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), 1.0, 0.0, False)
    b = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 2.5, 1e-4, inst=inst)
    for k in ("rgb", "alpha", "depth", "nsamp"):
        assert np.array_equal(a[k], b[k])


def test_instance_scale_and_rotation_invariance(oracle_lib):
    """Scaling the tree and the camera together keeps rgb/alpha and scales depth (opacity is
    measured in leaf units); a rotation of both is invisible."""
    from oracle.core import Instance
    sc = make_scene(5, 3000, "random", seed=5, T=10)
    o, d = random_rays(sc.G, 300, np.random.default_rng(6))
    o = (np.round(o * 256) / 256).astype(np.float32)   # coarse origins keep s*o + tr exact in float32
    # scale by a power of two and translate by integers: every float32 input stays exact
    s = 2.0
    tr = np.array([3.0, -5.0, 7.0], np.float32)
    inst = Instance(np.eye(3, dtype=np.float32), tr, s, 0.0, False)
    a = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, 1.0, 1e-4)
    b = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, (o * s + tr).astype(np.float32),
                          d, None, 1.0, 1e-4, inst=inst)
    assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-12
    assert np.abs(a["alpha"] - b["alpha"]).max() < 1e-12
    fin = np.isfinite(a["depth"])
    assert np.array_equal(fin, np.isfinite(b["depth"]))
    assert np.abs(a["depth"][fin] * s - b["depth"][fin]).max() < 1e-9
    # a quarter turn about z maps the grid onto itself; rotate the rays with it
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    Gc = sc.G
    tr2 = np.array([Gc, 0, 0], np.float32)   # world = R x_l + tr2 keeps the cube in place
    inst2 = Instance(R, tr2, 1.0, 0.0, False)
    ow = (o @ R.T + tr2).astype(np.float32)
    dw = (d @ R.T).astype(np.float32)
    c = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, ow, dw, None, 1.0, 1e-4, inst=inst2)
    assert np.abs(a["rgb"] - c["rgb"]).max() < 1e-12
    assert np.abs(a["alpha"] - c["alpha"]).max() < 1e-12


def test_pinhole_rays(oracle_lib):
    from workloads import orbit_camera
    cam = orbit_camera((10.0, 20.0, 30.0), 50.0, 0.7, 0.2, 64, 48, 60.0)
    o, d = oracle_lib.pinhole_rays(cam.width, cam.height, cam.intr(), cam.c2w)
    assert o.shape == (64 * 48, 3)
    assert np.all(o == cam.c2w[:, 3])
    assert np.abs(np.linalg.norm(d.astype(np.float64), axis=1) - 1).max() < 1e-6
    # the four central pixels straddle the optical axis symmetrically
    ctr = d.reshape(48, 64, 3)[23:25, 31:33].reshape(4, 3).astype(np.float64).mean(0)
    fwd = cam.c2w[:, 2].astype(np.float64)
    assert np.abs(ctr / np.linalg.norm(ctr) - fwd / np.linalg.norm(fwd)).max() < 1e-6
    # image x grows along the camera's right axis, image y along its down axis
    assert np.dot(d[1] - d[0], cam.c2w[:, 0]) > 0
    assert np.dot(d[64] - d[0], cam.c2w[:, 1]) > 0
    # pixel subset = same rays
    pix = np.array([0, 5, 64 * 47 + 63, 1000], np.int32)
    o2, d2 = oracle_lib.pinhole_rays(cam.width, cam.height, cam.intr(), cam.c2w, pix)
    assert np.array_equal(d2, d[pix]) and np.array_equal(o2, o[pix])


def test_pinhole_focal_scaling(oracle_lib):
    """Corner and edge pixels of a camera with fx != fy and an off-centre principal
    point: in the camera frame the ray of pixel (u, v) makes the angle
    atan((u + 1/2 - cx) / fx) with the optical axis in the x-z plane and
    atan((v + 1/2 - cy) / fy) in the y-z plane (OpenCV axes). Swapping fx and fy,
    dropping the half-pixel offset or the division by the focal length fails."""
    W, H = 40, 24
    fx, fy, cx, cy = 30.0, 55.0, 21.0, 11.5
    ang = 0.4
    R = np.array([[np.cos(ang), 0.0, np.sin(ang)], [0.0, 1.0, 0.0], [-np.sin(ang), 0.0, np.cos(ang)]])
    c2w = np.concatenate([R, np.array([[1.0], [-2.0], [3.0]])], axis=1).astype(np.float32)
    uv = [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (0, H // 2), (W - 1, H // 2), (W // 2, 0),
          (W // 2, H - 1)]
    pix = np.array([v * W + u for u, v in uv], np.int32)
    o, d = oracle_lib.pinhole_rays(W, H, (fx, fy, cx, cy), c2w, pix)
    dc = d.astype(np.float64) @ c2w[:, :3].astype(np.float64)    # camera frame: R^T d
    for i, (u, v) in enumerate(uv):
        ax = math.atan2(dc[i, 0], dc[i, 2])
        ay = math.atan2(dc[i, 1], dc[i, 2])
        assert abs(ax - math.atan((u + 0.5 - cx) / fx)) < 2e-7, (u, v)
        assert abs(ay - math.atan((v + 0.5 - cy) / fy)) < 2e-7, (u, v)
        # angle from the optical axis
        full = math.atan(math.hypot((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy))
        assert abs(math.acos(min(1.0, dc[i, 2] / np.linalg.norm(dc[i]))) - full) < 2e-6, (u, v)


# ---------------------------------------------------------------------------
# per-point hyperangle (Eq. 6): gamma = pi * sigmoid(sum_c wgam_c B_c(t))

def test_per_point_hyperangle_reduces_to_global_table(oracle_lib):
    sc = make_scene(5, 3000, "random", seed=13, T=10)
    o, d = random_rays(sc.G, 300, np.random.default_rng(14))
    wg = np.ones((sc.n_leaves, 1), np.float32)
    g = sc.gamma.astype(np.float64) / math.pi
    bg = np.log(g / (1 - g)).astype(np.float32)[:, None]     # logit: sigmoid(bg) * pi = gamma
    for t in (0.0, 3.0, 9.0):
        a = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma, o, d, None, t, 1e-4)
        b = oracle_lib.render(5, sc.leaf_ijk, sc.hh, sc.wsig, sc.basis, sc.gamma * 0 + 0.123, o, d, None, t, 1e-4,
                              wgam=wg, basis_g=bg)
        # basis_g holds float32 logits: gamma agrees to float32 rounding of the logit
        assert np.abs(a["rgb"] - b["rgb"]).max() < 1e-6
        assert np.abs(a["alpha"] - b["alpha"]).max() < 1e-14


@pytest.mark.parametrize("t_stop,seed", [(0.0, 21), (0.05, 22)])
def test_per_point_hyperangle_matches_bruteforce(oracle_lib, t_stop, seed):
    ijk, hh, wsig, basis, gamma = tiny_scene(3, seed=seed)
    rng = np.random.default_rng(seed + 1)
    wg = rng.normal(0, 1, (ijk.shape[0], 4)).astype(np.float32)
    bg = rng.normal(0, 1, (basis.shape[0], 4)).astype(np.float32)
    o1, d1 = random_rays(8, 40, rng, inside_frac=0.25)
    o2, d2 = special_rays(8)
    o = np.concatenate([o1, o2])
    d = np.concatenate([d1, d2])
    res = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, o, d, None, 3.0, t_stop, wgam=wg, basis_g=bg)
    for r in range(o.shape[0]):
        C, A, D, ns = BF.render(3, ijk, hh, wsig, basis, gamma, o[r].astype(np.float64), d[r].astype(np.float64),
                                3.0, t_stop, wgam=wg, basis_g=bg)
        assert np.allclose(res["rgb"][r], C, rtol=0, atol=1e-12), r
        assert abs(res["alpha"][r] - A) < 1e-12 and res["nsamp"][r] == ns, r


def test_per_point_hyperangle_gradient_finite_differences(oracle_lib):
    ijk, hh, wsig, basis, gamma = tiny_scene(3, n_leaves=60, seed=31, T=5)
    rng = np.random.default_rng(32)
    hh = hh.astype(np.float64)
    wg = rng.normal(0, 1, (60, 3))
    bg = rng.normal(0, 1, (5, 3))
    o, d = random_rays(8, 30, rng)
    t = rng.uniform(0, 4, 30).astype(np.float32)
    gC = rng.normal(size=(30, 3))
    gA = rng.normal(size=30)

    def run(hh_, wg_, bg_):
        r = oracle_lib.render(3, ijk, hh_, wsig, basis, gamma, o, d, t, 0.0, 0.0, g_rgb=gC, g_alpha=gA,
                              wgam=wg_, basis_g=bg_)
        return float((r["rgb"] * gC).sum() + (r["alpha"] * gA).sum()), r

    L0, res = run(hh, wg, bg)
    eps = 1e-6
    touched = np.unique(np.nonzero(np.abs(res["grad_wgam"]).sum(1))[0])
    assert touched.size > 5
    for q in touched[:6]:
        for c in range(3):
            a = wg.copy(); a[q, c] += eps
            b = wg.copy(); b[q, c] -= eps
            fd = (run(hh, a, bg)[0] - run(hh, b, bg)[0]) / (2 * eps)
            assert abs(fd - res["grad_wgam"][q, c]) < 1e-7 * max(1, abs(fd))
        a = hh.copy(); a[q, 1, 7] += eps
        b = hh.copy(); b[q, 1, 7] -= eps
        fd = (run(a, wg, bg)[0] - run(b, wg, bg)[0]) / (2 * eps)
        assert abs(fd - res["grad_hh"][q, 1, 7]) < 1e-7 * max(1, abs(fd))
    for i in range(5):
        for c in range(3):
            a = bg.copy(); a[i, c] += eps
            b = bg.copy(); b[i, c] -= eps
            fd = (run(hh, wg, a)[0] - run(hh, wg, b)[0]) / (2 * eps)
            assert abs(fd - res["grad_basis_g"][i, c]) < 1e-7 * max(1, abs(fd))


# ---------------------------------------------------------------------------
# ReLU density (Eq. 5 as printed): the same pins for the second activation

@pytest.mark.parametrize("depth,t_stop,seed", [(3, 0.0, 21), (4, 1e-3, 22)])
def test_relu_density_matches_bruteforce(oracle_lib, depth, t_stop, seed):
    ijk, hh, wsig, basis, gamma = tiny_scene(depth, seed=seed)
    G = 1 << depth
    rng = np.random.default_rng(seed + 100)
    o1, d1 = random_rays(G, 40, rng, inside_frac=0.25)
    o2, d2 = special_rays(G)
    o = np.concatenate([o1, o2])
    d = np.concatenate([d1, d2])
    res = oracle_lib.render(depth, ijk, hh, wsig, basis, gamma, o, d, None, 2.0, t_stop, density="relu")
    soft = oracle_lib.render(depth, ijk, hh, wsig, basis, gamma, o, d, None, 2.0, t_stop)
    assert np.abs(res["alpha"] - soft["alpha"]).max() > 1e-3   # the activation reaches the output
    for r in range(o.shape[0]):
        C, A, D, ns = BF.render(depth, ijk, hh, wsig, basis, gamma, o[r].astype(np.float64),
                                d[r].astype(np.float64), 2.0, t_stop, density="relu")
        assert np.allclose(res["rgb"][r], C, rtol=0, atol=1e-12), r
        assert abs(res["alpha"][r] - A) < 1e-12, r
        assert (math.isinf(D) and math.isinf(res["depth"][r])) or abs(res["depth"][r] - D) < 1e-9, r
        assert res["nsamp"][r] == ns, (r, res["nsamp"][r], ns)


def test_relu_single_voxel_closed_form(oracle_lib):
    """alpha = 1 - exp(-max(x, 0) l) exactly; a voxel with a negative logit is a composited sample of
    zero weight (transparent: no colour, no alpha, depth +inf)."""
    ijk = np.array([[1, 2, 3]], np.int32)
    hh = np.array([[[0.7], [-0.4], [1.3]]], np.float32)
    basis = np.array([[1.0, 2.0], [0.5, -1.0]], np.float32)
    gamma = np.array([0.4, 1.1], np.float32)
    h0 = 1.0 / (math.pi * math.sqrt(2.0))
    c = np.array([1 / (1 + math.exp(-float(v) * h0)) for v in hh[0, :, 0]])
    o, d, ell = (0.0, 1.0, 2.0), (1, 1, 1), math.sqrt(3.0)
    for wsig in (np.array([[0.9, -0.3]], np.float32), np.array([[0.25, 0.5]], np.float32),
                 np.array([[-0.9, 0.3]], np.float32)):
        x = float(wsig[0, 0]) * 1.0 + float(wsig[0, 1]) * 2.0
        res = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, np.array([o]), np.array([d]), None, 0.0, 0.0,
                                density="relu")
        a = 1 - math.exp(-max(x, 0.0) * ell)
        assert abs(res["alpha"][0] - a) < 1e-14
        assert np.abs(res["rgb"][0] - a * c).max() < 1e-14
        assert res["nsamp"][0] == 1
        if x < 0:
            assert res["alpha"][0] == 0.0 and np.all(res["rgb"][0] == 0.0) and math.isinf(res["depth"][0])


def test_relu_gradient_matches_finite_differences(oracle_lib):
    """Central differences of the ReLU-density loss, on rays and leaves whose density logits stay
    farther than the step from the kink at 0 (elsewhere the derivative is one-sided)."""
    ijk, hh, wsig, basis, gamma = tiny_scene(3, n_leaves=60, seed=13, T=5)
    hh = hh.astype(np.float64)
    wsig = wsig.astype(np.float64)
    basis = basis.astype(np.float64)
    rng = np.random.default_rng(14)
    o, d = random_rays(8, 30, rng)
    t = np.full(30, 2.0, np.float32)   # one frame: b = basis[2], so every logit is wsig . basis[2]
    x = wsig @ basis[2]
    far = np.abs(x) > 1e-3
    gC = rng.normal(size=(30, 3))
    gA = rng.normal(size=30)

    def loss(hh_, wsig_, basis_):
        r = oracle_lib.render(3, ijk, hh_, wsig_, basis_, gamma, o, d, t, 0.0, 0.0, g_rgb=gC, g_alpha=gA,
                              density="relu")
        return float((r["rgb"] * gC).sum() + (r["alpha"] * gA).sum()), r

    L0, res = loss(hh, wsig, basis)
    eps = 1e-6
    # leaves the rays sample (every sampled leaf has a colour gradient with the softplus density)
    soft = oracle_lib.render(3, ijk, hh, wsig, basis, gamma, o, d, t, 0.0, 0.0, g_rgb=gC, g_alpha=gA)
    visited = np.unique(np.nonzero(np.abs(soft["grad_hh"]).sum((1, 2)))[0])
    # sampled leaves with a negative logit are transparent: no gradient to their colour or density
    neg = visited[x[visited] < 0]
    assert neg.size > 3
    assert np.all(res["grad_wsig"][neg] == 0.0) and np.all(res["grad_hh"][neg] == 0.0)
    touched = visited[x[visited] > 0]
    assert touched.size > 5
    checked = 0
    for q in touched[:10]:
        if not far[q]:
            continue
        for idx in ((q, 0, 0), (q, 2, 15)):
            a = hh.copy(); a[idx] += eps
            b = hh.copy(); b[idx] -= eps
            fd = (loss(a, wsig, basis)[0] - loss(b, wsig, basis)[0]) / (2 * eps)
            assert abs(fd - res["grad_hh"][idx]) < 1e-7 * max(1, abs(res["grad_hh"][idx]))
        for cc in range(wsig.shape[1]):
            a = wsig.copy(); a[q, cc] += eps
            b = wsig.copy(); b[q, cc] -= eps
            fd = (loss(hh, a, basis)[0] - loss(hh, b, basis)[0]) / (2 * eps)
            assert abs(fd - res["grad_wsig"][q, cc]) < 1e-7 * max(1, abs(res["grad_wsig"][q, cc]))
        checked += 1
    assert checked >= 4
    # basis row 2 (the only one used): every logit moves with it; keep the step below the
    # smallest distance of a touched logit from the kink
    step = min(eps, 0.1 * np.abs(x[touched]).min())
    for cc in (0, 5):
        a = basis.copy(); a[2, cc] += step
        b = basis.copy(); b[2, cc] -= step
        fd = (loss(hh, wsig, a)[0] - loss(hh, wsig, b)[0]) / (2 * step)
        assert abs(fd - res["grad_basis"][2, cc]) < 1e-6 * max(1, abs(res["grad_basis"][2, cc]))

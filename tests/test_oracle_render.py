"""Pins of the oracle's projection, SH colour, sort, blend (Eq. 1, Eq. 2) and
backward against closed forms, library routines and finite differences."""
import math

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import configs

from _helpers import single_splat_tree

C0 = 0.28209479177387814


def _ulp_dist(a32: np.ndarray, ref64: np.ndarray) -> np.ndarray:
    ulp = np.spacing(np.abs(ref64).astype(np.float32)).astype(np.float64)
    return np.abs(a32.astype(np.float64) - ref64) / ulp


def test_portable_exp_within_2ulp():
    xs = np.concatenate([np.linspace(-87.0, 0.0, 20001), np.linspace(0.0, 20.0, 2001),
                         np.random.default_rng(0).uniform(-87, 20, 20000)]).astype(np.float32)
    got = oracle.pexp(xs)
    ref = np.exp(xs.astype(np.float64))
    assert _ulp_dist(got, ref).max() <= 2.0
    assert oracle.pexp(np.float32(-87.5)) == 0 and oracle.pexp(np.float32(-np.inf)) == 0


def test_sh_basis_matches_scipy_real_harmonics():
    """Real SH (l <= 3) built from SciPy's complex Y_l^m; each basis function must
    equal it up to one fixed sign (the Condon-Shortley convention)."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(1)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta, phi = np.arccos(d[:, 2]), np.arctan2(d[:, 1], d[:, 0])
    ours = np.array([oracle.sh_basis(v) for v in d])
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                real = math.sqrt(2) * (-1) ** m * Y.real
            elif m < 0:
                real = math.sqrt(2) * (-1) ** m * Y.imag
            else:
                real = Y.real
            k = l * l + l + m
            s = np.sign(np.dot(ours[:, k], real))
            assert s != 0
            np.testing.assert_allclose(ours[:, k], s * real, rtol=0, atol=1e-12)


def test_sh_basis_gradient_by_finite_differences():
    rng = np.random.default_rng(2)
    for _ in range(20):
        d = rng.normal(size=3)
        _, dY = oracle.sh_basis(d, with_grad=True)
        h = 1e-6
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (oracle.sh_basis(d + e) - oracle.sh_basis(d - e)) / (2 * h)
            np.testing.assert_allclose(dY[:, a], fd, rtol=1e-6, atol=1e-8)


def _cam64(w=64, h=64, dist=10.0):
    return scenegen.camera_look_at((0.0, 0.0, dist), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), w, h)


def test_projection_on_axis_isotropic_closed_form():
    cam = _cam64()
    s = 0.2
    P = np.zeros(11 + 3)
    P[3:6] = math.log(s)
    P[6] = 1.0
    P[10] = 0.3
    P[11:14] = (np.array([0.2, 0.4, 0.9]) - 0.5) / C0
    out = oracle.project64_one(P, 3, cam)
    f = cam.fx
    var = (f * s / 10.0) ** 2 + 0.3
    np.testing.assert_allclose(out[[0, 1]], [cam.cx, cam.cy], atol=1e-9)
    np.testing.assert_allclose(out[[2, 3, 4]], [var, 0.0, var], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out[[5, 6, 7]], [1 / var, 0.0, 1 / var], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out[8], 1 / (1 + math.exp(-0.3)), rtol=1e-14)
    np.testing.assert_allclose(out[9:12], [0.2, 0.4, 0.9], rtol=1e-12)


def test_projection_matches_numerical_jacobian_and_scipy_rotation():
    """EWA: Sigma' = J W Sigma W^T J^T + 0.3 I with J the derivative of the pinhole
    map (taken numerically here) and Sigma from SciPy's quaternion rotation."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(3)
    for _ in range(50):
        cam = scenegen.camera_look_at(rng.uniform(-20, 20, 3) + [0, 0, 30], rng.uniform(-2, 2, 3), (0, 1, 0),
                                      96, 64, hfov_deg=rng.uniform(40, 80))
        P = np.zeros(11 + 3)
        P[0:3] = rng.uniform(-3, 3, 3)
        P[3:6] = rng.normal(-1, 0.5, 3)
        P[6:10] = rng.normal(size=4) * rng.uniform(0.5, 2)
        P[10] = rng.normal()
        out = oracle.project64_one(P, 3, cam)
        R = cam.R.astype(np.float64)
        c = R @ P[0:3] + cam.t.astype(np.float64)
        pin = lambda v: np.array([cam.fx * v[0] / v[2] + cam.cx, cam.fy * v[1] / v[2] + cam.cy])
        J = np.zeros((2, 3))
        for a in range(3):
            e = np.zeros(3)
            e[a] = 1e-6
            J[:, a] = (pin(c + e) - pin(c - e)) / 2e-6
        qn = P[6:10] / np.linalg.norm(P[6:10])
        Rq = Rotation.from_quat([qn[1], qn[2], qn[3], qn[0]]).as_matrix()
        Sig = Rq @ np.diag(np.exp(2 * P[3:6])) @ Rq.T
        Sp = J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(out[[0, 1]], pin(c), rtol=1e-12)
        np.testing.assert_allclose(out[[2, 3, 4]], [Sp[0, 0], Sp[0, 1], Sp[1, 1]], rtol=1e-6)
        con = np.array([[out[5], out[6]], [out[6], out[7]]])
        np.testing.assert_allclose(con @ np.array([[out[2], out[3]], [out[3], out[4]]]), np.eye(2), atol=1e-10)
        assert out[12] == pytest.approx(c[2])


def test_tile_rectangle_matches_bruteforce_square_intersection(tiny_tree, tiny_oracle):
    cam = configs.tiny_camera()
    ids, _ = tiny_oracle.select(cam, 4.0)
    F = oracle.OracleFrame(tiny_tree, ids, cam)
    sp = F.splats()
    TX = TY = 32
    txs = np.arange(TX)
    for i in range(0, len(ids), 7):
        f = sp["f32"][i].astype(np.float64)
        mx, my, r = f[0] + f[1], f[2] + f[3], f[9]
        if r == 0:
            continue
        xs = txs[(txs * 16 <= mx + r) & ((txs + 1) * 16 > mx - r)]
        ys = txs[(txs * 16 <= my + r) & ((txs + 1) * 16 > my - r)]
        x0, x1, y0, y1 = sp["rect"][i]
        if len(xs) and len(ys):
            assert (x0, x1, y0, y1) == (xs.min(), xs.max() + 1, ys.min(), ys.max() + 1)
            assert sp["tiles"][i] == len(xs) * len(ys)
        else:
            assert sp["tiles"][i] == 0


def test_instance_order_is_stable_sort_of_tile_depth_keys(tiny_tree, tiny_oracle):
    cam = configs.tiny_camera()
    ids, _ = tiny_oracle.select(cam, 2.0)
    F = oracle.OracleFrame(tiny_tree, ids, cam)
    sp = F.splats()
    tile, pos, depth = [], [], []
    for i in range(len(ids)):
        x0, x1, y0, y1 = sp["rect"][i]
        if sp["tiles"][i] == 0:
            continue
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                tile.append(ty * 32 + tx)
                pos.append(i)
                depth.append(sp["depth_bits"][i])
    key = (np.array(tile, np.uint64) << np.uint64(32)) | np.array(depth, np.uint64)
    order = np.argsort(key, kind="stable")
    t2, p2 = F.instances()
    assert np.array_equal(t2, np.array(tile)[order]) and np.array_equal(p2, np.array(pos)[order])


def _f32(v):
    """Value after the FP32 storage of a parameter."""
    return np.float64(np.float32(v))


def _eff(s, o, rgb):
    """Scale, opacity and colour as the FP32-stored parameters encode them."""
    s_e = math.exp(_f32(math.log(s)))
    lg = _f32(math.log(o / (1 - o)))
    o_e = 1 / (1 + math.exp(-lg))
    rgb_e = 0.5 + C0 * np.array([_f32((c - 0.5) / C0) for c in rgb])
    return s_e, o_e, rgb_e


def _alpha_on_axis(o, var, shape, center):
    ys, xs = np.mgrid[0:shape[0], 0:shape[1]]
    d2 = (xs + 0.5 - center[0]) ** 2 + (ys + 0.5 - center[1]) ** 2
    return np.minimum(0.99, o * np.exp(-0.5 * d2 / var))


def test_single_gaussian_image_closed_form():
    cam = _cam64()
    o = 0.3  # alpha = 1/255 lies inside the 3-sigma footprint for o <= 0.3
    s = 0.15
    rgb = np.array([0.9, 0.5, 0.2])
    t = single_splat_tree([dict(mean=(0, 0, 0), log_scale=(math.log(s),) * 3, logit=math.log(o / (1 - o)),
                                rgb=rgb)])
    F = oracle.OracleFrame(t, np.array([0]), cam)
    s, o, rgb = _eff(s, o, rgb)
    var = (cam.fx * s / 10.0) ** 2 + 0.3
    a = _alpha_on_axis(o, var, (64, 64), (cam.cx, cam.cy))
    safe = np.abs(a - 1 / 255) > 1e-6
    expect = np.where(a >= 1 / 255, a, 0.0)[..., None] * rgb
    np.testing.assert_allclose(F.image[safe], expect[safe], rtol=1e-12, atol=1e-14)
    assert F.image.max() > 0.15


def test_two_gaussian_compositing_and_depth_swap():
    cam = _cam64()
    rgb1, rgb2 = np.array([1.0, 0.1, 0.1]), np.array([0.1, 0.2, 1.0])
    o1, o2, s1, s2 = 0.25, 0.3, 0.2, 0.12

    def scene(z1, z2):
        return single_splat_tree([
            dict(mean=(0, 0, z1), log_scale=(math.log(s1),) * 3, logit=math.log(o1 / (1 - o1)), rgb=rgb1),
            dict(mean=(0, 0, z2), log_scale=(math.log(s2),) * 3, logit=math.log(o2 / (1 - o2)), rgb=rgb2)])

    for z1, z2 in ((0.0, -2.0), (-2.0, 0.0)):
        t = scene(z1, z2)
        F = oracle.OracleFrame(t, np.array([0, 1]), cam)
        d1, d2 = 10.0 - z1, 10.0 - z2
        e1, q1, c1 = _eff(s1, o1, rgb1)
        e2, q2, c2 = _eff(s2, o2, rgb2)
        a1 = _alpha_on_axis(q1, (cam.fx * e1 / d1) ** 2 + 0.3, (64, 64), (cam.cx, cam.cy))
        a2 = _alpha_on_axis(q2, (cam.fx * e2 / d2) ** 2 + 0.3, (64, 64), (cam.cx, cam.cy))
        safe = (np.abs(a1 - 1 / 255) > 1e-6) & (np.abs(a2 - 1 / 255) > 1e-6)
        a1 = np.where(a1 >= 1 / 255, a1, 0.0)[..., None]
        a2 = np.where(a2 >= 1 / 255, a2, 0.0)[..., None]
        if d1 < d2:
            expect = c1 * a1 + c2 * a2 * (1 - a1)
        else:
            expect = c2 * a2 + c1 * a1 * (1 - a2)
        np.testing.assert_allclose(F.image[safe], expect[safe], rtol=1e-12, atol=1e-14)


def test_early_termination_stops_before_transmittance_drops_below_1e4():
    cam = _cam64()
    o = 0.8
    rgb = np.array([0.3, 0.6, 0.9])
    t = single_splat_tree([dict(mean=(0, 0, -k), log_scale=(math.log(1.0),) * 3, logit=math.log(o / (1 - o)),
                                rgb=rgb) for k in range(6)])
    F = oracle.OracleFrame(t, np.arange(6), cam)
    counts = F.pixel_counts()
    assert counts[31, 31] == 5  # T after 5 splats ~ 3.4e-4, the 6th would give ~6.8e-5
    s_e, o, rgb = _eff(1.0, o, rgb)
    a = [o * math.exp(-0.5 * 0.5 / ((cam.fx * s_e / (10.0 + k)) ** 2 + 0.3)) for k in range(5)]
    T, C = 1.0, np.zeros(3)
    for ak in a:
        C += rgb * ak * T
        T *= 1 - ak
    np.testing.assert_allclose(F.image[31, 31], C, rtol=1e-12)


def test_weights_sum_to_one_minus_final_transmittance(tiny_tree, tiny_oracle):
    """With every colour 1 and background 1 each pixel is sum_i a_i T_i + T_final = 1;
    with background 0 it is 1 - T_final, in [0, 1]."""
    cam = configs.tiny_camera(128, 128)
    ids, _ = tiny_oracle.select(cam, 1.0)
    t = tiny_tree
    white = scenegen.Tree(t.n_leaves, t.sh_degree, t.means, t.log_scales, t.quats, t.opacity_logits,
                          np.zeros_like(t.sh), t.left, t.right, t.parent, t.root, t.log_volume_threshold)
    white.sh[:, 0, :] = 0.5 / C0
    F1 = oracle.OracleFrame(white, ids, cam, bg=(1.0, 1.0, 1.0))
    np.testing.assert_allclose(F1.image, 1.0, atol=1e-12)
    F0 = oracle.OracleFrame(white, ids, cam)
    assert F0.image.min() >= 0 and F0.image.max() <= 1.0 + 1e-12 and F0.image.max() > 0.5


def test_backward_matches_central_differences_with_frozen_decisions():
    rng = np.random.default_rng(4)
    n = 24
    params = []
    for _ in range(n):
        params.append(dict(mean=rng.uniform(-1.5, 1.5, 3), log_scale=rng.normal(-1.2, 0.3, 3),
                           quat=rng.normal(size=4), logit=rng.normal(), rgb=rng.uniform(0.6, 0.9, 3),
                           sh=rng.normal(0, 0.05, (15, 3))))
    t = single_splat_tree(params, sh_degree=3)
    cam = scenegen.camera_look_at((0.7, -0.5, 8.0), (0, 0, 0), (0, 1, 0), 48, 40)
    F = oracle.OracleFrame(t, np.arange(n), cam)
    dL = rng.normal(size=F.image.shape)
    g2, g = F.backward(dL)
    P0 = F.params64()
    fd = np.zeros_like(g)
    for i in range(n):
        for k in range(P0.shape[1]):
            h = 1e-6 * max(1.0, abs(P0[i, k]))
            P = P0.copy()
            P[i, k] += h
            up = np.sum(dL * F.eval_frozen(P))
            P[i, k] -= 2 * h
            dn = np.sum(dL * F.eval_frozen(P))
            fd[i, k] = (up - dn) / (2 * h)
    groups = {"mean": slice(0, 3), "log_scale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
              "sh": slice(11, None)}
    for name, sl in groups.items():
        a, b = g[:, sl], fd[:, sl]
        scale = np.abs(b).max()
        assert scale > 0, name
        assert np.abs(a - b).max() <= 1e-6 * scale, (name, np.abs(a - b).max(), scale)


def test_directional_fd_matches_full_reevaluation_and_backward():
    """The local directional difference (only the splat's pixels recomposited)
    equals the full frozen re-evaluation and the analytic gradient."""
    rng = np.random.default_rng(9)
    n = 16
    params = [dict(mean=rng.uniform(-1.5, 1.5, 3), log_scale=rng.normal(-1.2, 0.3, 3), quat=rng.normal(size=4),
                   logit=rng.normal(), rgb=rng.uniform(0.6, 0.9, 3), sh=rng.normal(0, 0.05, (15, 3)))
              for _ in range(n)]
    t = single_splat_tree(params, sh_degree=3)
    cam = scenegen.camera_look_at((0.4, -0.3, 8.0), (0, 0, 0), (0, 1, 0), 40, 32)
    F = oracle.OracleFrame(t, np.arange(n), cam)
    W = rng.normal(size=F.image.shape)
    _, g = F.backward(W)
    P0 = F.params64()
    h = 1e-6
    for i in range(n):
        v = rng.normal(size=P0.shape[1])
        local = F.fd_directional(W, i, v, h)
        P = P0.copy()
        P[i] += h * v
        up = np.sum(W * F.eval_frozen(P))
        P[i] -= 2 * h * v
        dn = np.sum(W * F.eval_frozen(P))
        full = (up - dn) / (2 * h)
        assert abs(local - full) <= 1e-7 * max(1.0, abs(full))
        assert abs(local - g[i] @ v) <= 1e-6 * max(1e-3, np.abs(g[i]).max() * np.abs(v).max())


def test_splat_contribution_counts_closed_form():
    # one splat: it is composited into exactly the pixels where o e^power >=
    # 1/255 (nothing stops: 1 - alpha >= 0.01); two splats side by side along x
    # do not overlap: each count is its own disc
    cam = _cam64()
    o, s = 0.3, 0.15
    t = single_splat_tree([dict(mean=(0, 0, 0), log_scale=(math.log(s),) * 3, logit=math.log(o / (1 - o)),
                                rgb=(0.5, 0.5, 0.5))])
    F = oracle.OracleFrame(t, np.array([0]), cam)
    se, oe, _ = _eff(s, o, (0.5, 0.5, 0.5))
    a = _alpha_on_axis(oe, (cam.fx * se / 10.0) ** 2 + 0.3, (64, 64), (cam.cx, cam.cy))
    assert np.all(np.abs(a - 1 / 255) > 1e-6), "no pixel centre on the threshold"
    want = int((a >= 1 / 255).sum())
    assert want > 20
    assert F.splat_contrib().tolist() == [want]
    assert int(F.pixel_counts().sum()) == want
    # two splats 2.5 units apart on x (about 80 px): disjoint discs
    t2 = single_splat_tree([dict(mean=(-1.25, 0, 0), log_scale=(math.log(s),) * 3, logit=math.log(o / (1 - o)),
                                 rgb=(0.5, 0.5, 0.5)),
                            dict(mean=(1.25, 0, 0), log_scale=(math.log(s),) * 3, logit=math.log(o / (1 - o)),
                                 rgb=(0.5, 0.5, 0.5))])
    cam2 = _cam64(w=256, h=64)
    F2 = oracle.OracleFrame(t2, np.array([0, 1]), cam2)
    var = (cam2.fx * se / 10.0) ** 2 + 0.3
    counts = []
    for mx in (-1.25, 1.25):
        a = _alpha_on_axis(oe, var, (64, 256), (cam2.cx + cam2.fx * mx / 10.0, cam2.cy))
        assert np.all(np.abs(a - 1 / 255) > 1e-6)
        counts.append(int((a >= 1 / 255).sum()))
    assert F2.splat_contrib().tolist() == counts


def test_splat_contribution_counts_sum_to_the_contributor_lists(tiny_tree, tiny_oracle):
    cam = configs.tiny_camera(128, 128)
    ids, _ = tiny_oracle.select(cam, 1.0)
    F = oracle.OracleFrame(tiny_tree, ids, cam)
    c = F.splat_contrib()
    assert int(c.sum()) == F.info()["n_contrib"] == int(F.pixel_counts().sum())
    # a splat that is not drawn is composited nowhere
    assert np.all(c[F.splats()["tiles"] == 0] == 0)

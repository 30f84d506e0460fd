"""Pins of the oracle's FP32 decision record (the per-splat record behind every
alpha skip, clamp and termination: projected mean as a hi/lo pair, principal
axis (ce, se), power coefficients h1 = -1/(2 l1), h2 = -1/(2 l2), footprint
radius, opacity) and of its FP64-disagreement log.

The record is checked against quantities derived independently of it: the
eigen-decomposition (numpy.linalg.eigh) of the FP64 projected covariance of
Sec. 3's EWA projection (itself pinned against SciPy's rotation and a
numerical Jacobian), the FP64 conic power -d^T Sigma'^-1 d / 2 at sampled
pixels, and a closed-form image of one rotated anisotropic splat.  The flip
counters are checked against closed-form FP64 alphas and compositing over
parameter sweeps that straddle each threshold."""
import math

import numpy as np
import pytest

import oracle
import scenegen

from _helpers import single_splat_tree

C0 = 0.28209479177387814


def _random_splats(rng, n, centre, spread, ls_lo, ls_hi, flat=False):
    out = []
    for _ in range(n):
        ls = rng.uniform(ls_lo, ls_hi, 3)
        if flat:
            ls[2] = ls_lo - 3.0  # a flat splat: one axis much thinner
        out.append(dict(mean=np.asarray(centre) + rng.uniform(-spread, spread, 3) * np.array([1, 1, 0.0 if flat else 1]),
                        log_scale=ls, quat=rng.normal(size=4) * rng.uniform(0.5, 2.0), logit=rng.normal(),
                        rgb=rng.uniform(0.2, 0.8, 3)))
    return out


def _cases():
    rng = np.random.default_rng(21)
    yield "regular", _random_splats(rng, 300, (0, 0, 0), 5.0, -3.0, 0.0), \
        scenegen.camera_look_at((0, 0, 30), (0, 0, 0), (0, 1, 0), 256, 192)
    # a camera just above a plane of flat splats, looking along it: needles
    yield "grazing", _random_splats(rng, 300, (0, 20, 0), 15.0, -2.0, 0.5, flat=True), \
        scenegen.camera_look_at((0, -5, 0.4), (0, 30, 0.0), (0, 0, 1), 320, 180)
    # splats just beyond the near plane (0.2): very large projected covariances
    near = []
    for _ in range(200):
        d = rng.uniform(0.22, 0.8)
        p = _random_splats(rng, 1, (0, 0, 0), 0.0, -2.5, -0.5)[0]
        p["mean"] = np.array([rng.uniform(-0.3, 0.3) * d, rng.uniform(-0.3, 0.3) * d, 10.0 - d])
        near.append(p)
    yield "near-plane", near, scenegen.camera_look_at((0, 0, 10), (0, 0, 0), (0, 1, 0), 200, 200)


def _records(params, cam):
    t = single_splat_tree(params)
    F = oracle.OracleFrame(t, np.arange(len(params)), cam)
    sp = F.splats()
    P = F.params64()
    rec = sp["f32"].astype(np.float64)
    vals = np.array([oracle.project64_one(P[i], 3, cam) for i in range(len(params))])
    keep = rec[:, 9] > 0  # the record is formed for splats past the near plane with det > 0
    return rec[keep], vals[keep], P[keep]


@pytest.mark.parametrize("name,params,cam", list(_cases()), ids=[c[0] for c in _cases()])
def test_record_against_eigen_decomposition(name, params, cam):
    rec, vals, P = _records(params, cam)
    assert len(rec) >= 100, name
    mxh, mxl, myh, myl, ce, se, h1, h2, o, rad = rec.T
    mx, my, A, B, Cc, ca, cb, cc = vals[:, :8].T
    l_small, l_big, v_big = [], [], []
    for a, b, c in zip(A, B, Cc):
        w, V = np.linalg.eigh(np.array([[a, b], [b, c]]))
        l_small.append(w[0])
        l_big.append(w[1])
        v_big.append(V[:, 1])
    l_small, l_big, v_big = np.array(l_small), np.array(l_big), np.array(v_big)
    aniso = l_big / l_small
    assert aniso.max() > {"regular": 20.0, "grazing": 1000.0, "near-plane": 10.0}[name], (name, aniso.max())
    # the record's chain takes its scales from the FP32 exp: ~1e-7 relative
    np.testing.assert_allclose(h1, -0.5 / l_big, rtol=2e-6)
    np.testing.assert_allclose(h2, -0.5 / l_small, rtol=2e-6)
    np.testing.assert_allclose(ce * ce + se * se, 1.0, atol=1e-6)
    sep = (l_big - l_small) / l_big > 1e-3  # a well defined principal axis
    assert sep.sum() > 0.9 * len(sep)
    align = np.abs(ce * v_big[:, 0] + se * v_big[:, 1])
    assert np.all(align[sep] >= 1.0 - 1e-6), (name, align[sep].min())
    # mean: hi/lo pair of the FP64 projected mean
    np.testing.assert_allclose(mxh + mxl, mx, rtol=0, atol=1e-9 * np.maximum(1.0, np.abs(mx)).max())
    np.testing.assert_allclose(myh + myl, my, rtol=0, atol=1e-9 * np.maximum(1.0, np.abs(my)).max())
    np.testing.assert_allclose(o, 1.0 / (1.0 + np.exp(-P[:, 10])), rtol=1e-6)
    # footprint: ceil(3 sqrt(lambda_max)), lambda_max with the discriminant floored at 0.1
    mid, half = 0.5 * (l_big + l_small), 0.5 * (l_big - l_small)
    r3 = 3.0 * np.sqrt(mid + np.maximum(math.sqrt(0.1), half))
    safe = np.abs(r3 - np.round(r3)) > 1e-5 * r3
    assert np.array_equal(rad[safe], np.ceil(r3[safe])), name
    # the power the record defines equals the FP64 conic power at sampled pixels
    rng = np.random.default_rng(5)
    for i in range(len(rec)):
        sig = 3.0 * math.sqrt(l_big[i])
        d = rng.uniform(-sig, sig, (16, 2))
        dx, dy = d[:, 0], d[:, 1]
        u1 = ce[i] * dx + se[i] * dy
        u2 = -se[i] * dx + ce[i] * dy
        p_rec = h1[i] * u1 * u1 + h2[i] * u2 * u2
        p64 = -0.5 * (ca[i] * dx * dx + 2.0 * cb[i] * dx * dy + cc[i] * dy * dy)
        scale = np.abs(h1[i]) * u1 * u1 + np.abs(h2[i]) * u2 * u2 + 1e-30
        assert np.all(np.abs(p_rec - p64) <= 1e-5 * scale + 1e-12), (name, i)


def _eff_scalar(v):
    return float(np.float32(v))


def test_rotated_anisotropic_single_gaussian_image_closed_form():
    """One rotated, anisotropic splat at the origin, camera on the z axis: at
    c = (0, 0, d) the EWA Jacobian is (f/d) [I2 | 0], so Sigma' = (f/d)^2
    (W Sigma W^T)[:2, :2] + 0.3 I with Sigma from SciPy's rotation; every
    pixel is rgb min(0.99, o exp(-dp^T Sigma'^-1 dp / 2)) where that alpha is
    at least 1/255."""
    from scipy.spatial.transform import Rotation
    W_, H_ = 128, 96
    dist = 5.0
    cam = scenegen.camera_look_at((0, 0, dist), (0, 0, 0), (0, 1, 0), W_, H_)
    ls = np.array([math.log(0.5), math.log(0.04), math.log(0.1)])
    quat = Rotation.from_euler("zyx", [32.0, 17.0, -11.0], degrees=True).as_quat()  # (x, y, z, w)
    q = np.array([quat[3], quat[0], quat[1], quat[2]])
    o_target, rgb = 0.28, np.array([0.8, 0.4, 0.3])
    t = single_splat_tree([dict(mean=(0, 0, 0), log_scale=ls, quat=q, logit=math.log(o_target / (1 - o_target)),
                                rgb=rgb)])
    F = oracle.OracleFrame(t, np.array([0]), cam)
    # effective (FP32-stored) parameters
    s = np.exp(t.log_scales[0].astype(np.float64))
    qf = t.quats[0].astype(np.float64)
    o = 1.0 / (1.0 + math.exp(-float(t.opacity_logits[0])))
    rgb_e = 0.5 + C0 * t.sh[0, 0].astype(np.float64)
    Rq = Rotation.from_quat([qf[1], qf[2], qf[3], qf[0]]).as_matrix()
    Sig = Rq @ np.diag(s * s) @ Rq.T
    Wr = cam.R.astype(np.float64)
    Sc = Wr @ Sig @ Wr.T
    f = float(np.float32(cam.fx))
    cz = float(cam.R.astype(np.float64)[2] @ np.zeros(3) + cam.t.astype(np.float64)[2])
    Sp = (f / cz) ** 2 * Sc[:2, :2] + 0.3 * np.eye(2)
    Q = np.linalg.inv(Sp)
    ev = np.linalg.eigvalsh(Sp)
    assert ev[1] / ev[0] > 20.0  # anisotropic on screen
    assert abs(Sp[0, 1]) > 0.2 * math.sqrt(Sp[0, 0] * Sp[1, 1])  # and rotated
    ys, xs = np.mgrid[0:H_, 0:W_]
    dx, dy = xs + 0.5 - cam.cx, ys + 0.5 - cam.cy
    pw = -0.5 * (Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy)
    a = np.minimum(0.99, o * np.exp(pw))
    safe = np.abs(a - 1 / 255) > 1e-6
    expect = np.where(a >= 1 / 255, a, 0.0)[..., None] * rgb_e
    assert (a >= 1 / 255).sum() > 200
    np.testing.assert_allclose(F.image[safe], expect[safe], rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------ flip log
def _flip_sweep(make_params, thetas, cam, expected_fn):
    """Renders one frame per theta; returns (oracle's summed counters,
    closed-form summed counters)."""
    got = {"skip_flip64": 0, "stop_flip64": 0, "clamp_flip64": 0}
    want = {"skip_flip64": 0, "stop_flip64": 0, "clamp_flip64": 0}
    for th in thetas:
        params = make_params(th)
        t = single_splat_tree(params)
        F = oracle.OracleFrame(t, np.arange(len(params)), cam)
        info = F.info()
        for k in got:
            got[k] += info[k]
        for k, v in expected_fn(t, F).items():
            want[k] += v
    return got, want


def _alpha64(t, i, cam, shape):
    """FP64 o e^power of splat i of an on-axis scene (isotropic, mean on the
    optical axis at depth 10 - z) at every pixel, from closed form."""
    s = math.exp(float(t.log_scales[i, 0]))
    z = float(t.means[i, 2])
    var = (float(np.float32(cam.fx)) * s / (10.0 - z)) ** 2 + 0.3
    o = 1.0 / (1.0 + math.exp(-float(t.opacity_logits[i])))
    ys, xs = np.mgrid[0:shape[0], 0:shape[1]]
    d2 = (xs + 0.5 - cam.cx) ** 2 + (ys + 0.5 - cam.cy) ** 2
    return o * np.exp(-0.5 * d2 / var)


def _fine_thetas(center, n):
    """n consecutive FP32 values from center (as float64)."""
    v = np.float32(center)
    out = []
    for _ in range(n):
        out.append(float(v))
        v = np.nextafter(v, np.float32(np.inf))
    return out


def _logit_at(alpha_target, t, i, cam, shape, y, x):
    """The opacity logit that gives splat i the FP64 alpha alpha_target at
    pixel (y, x) (closed form), all else as in the tree t."""
    e = _alpha64(t, i, cam, shape)[y, x] * (1.0 + math.exp(-float(t.opacity_logits[i])))
    o = alpha_target / e
    return math.log(o / (1.0 - o))


def test_skip_flips_equal_closed_form_decisions():
    """One splat; over a sweep of opacity logits, in FP32 steps, around the
    logit where the closed-form FP64 alpha of the central pixels is exactly
    1/255, the oracle's count of skip decisions that FP64 takes the other way
    equals the count from the closed-form FP64 alpha against the FP32
    mirror's observed decision (a pixel contributes or not)."""
    W_ = 48
    cam = scenegen.camera_look_at((0, 0, 10), (0, 0, 0), (0, 1, 0), W_, W_)
    s = 0.08

    def mk(th):
        return [dict(mean=(0, 0, 0), log_scale=(math.log(s),) * 3, logit=th, rgb=(0.5, 0.5, 0.5))]

    def expected(t, F):
        a = np.minimum(0.99, _alpha64(t, 0, cam, (W_, W_)))
        fp32_hit = F.pixel_counts() > 0
        fp64_hit = a >= 1.0 / 255.0
        assert np.all(np.abs(a - 1.0 / 255.0) > 1e-15)  # no case the closed form cannot decide
        return {"skip_flip64": int((fp32_hit != fp64_hit).sum())}

    t0 = single_splat_tree(mk(0.0))
    thetas = []
    for (y, x) in ((24, 24), (24, 25), (25, 25)):  # d^2 = 0.5, 2.5, 4.5 from the principal point
        thetas += _fine_thetas(_logit_at(1.0 / 255.0, t0, 0, cam, (W_, W_), y, x) - 40 * 2.4e-7, 80)
    got, want = _flip_sweep(mk, thetas, cam, expected)
    assert got["skip_flip64"] == want["skip_flip64"]
    assert got["skip_flip64"] > 0, "the sweep never straddles the skip threshold"


def test_clamp_flips_equal_closed_form_decisions():
    """Opacity near the 0.99 clamp: the oracle's clamp flips equal those of the
    closed form (FP64 o e^power > 0.99) against the mirror's clamp, observed in
    the FP64 image (a clamped pixel is exactly 0.99 rgb)."""
    W_ = 32
    cam = scenegen.camera_look_at((0, 0, 10), (0, 0, 0), (0, 1, 0), W_, W_)
    s = 6.0  # wide: e^power stays close to 1 near the centre, so o e^power can reach 0.99
    rgb = np.array([0.7, 0.7, 0.7])

    def mk(th):
        return [dict(mean=(0, 0, 0), log_scale=(math.log(s),) * 3, logit=th, rgb=rgb)]

    def expected(t, F):
        e = _alpha64(t, 0, cam, (W_, W_))
        rgb_e = 0.5 + C0 * float(t.sh[0, 0, 0])
        clamped32 = F.image[..., 0] == 0.99 * rgb_e
        return {"clamp_flip64": int((clamped32 != (e > 0.99)).sum())}

    t0 = single_splat_tree(mk(0.0))
    thetas = []
    for (y, x) in ((16, 16), (16, 17)):
        thetas += _fine_thetas(_logit_at(0.99, t0, 0, cam, (W_, W_), y, x) - 60 * 4.8e-7, 120)
    got, want = _flip_sweep(mk, thetas, cam, expected)
    assert got["clamp_flip64"] == want["clamp_flip64"]
    assert got["clamp_flip64"] > 0


def test_stop_flips_equal_closed_form_decisions():
    """Three wide splats of alpha about 0.9 in front bring T to about 1e-3 near
    the centre; a fourth, smaller one puts T (1 - alpha) next to 1e-4 there.
    Its opacity is close to 1, so one FP32 step of its logit moves
    T (1 - alpha) by about 1e-9 relative, finer than the FP32 rounding of the
    test.  Its stop decision in FP64 (T the FP64 product along the mirror's
    decisions) against the mirror's (a pixel stops at the fourth splat: three
    contributors) gives the oracle's stop flips."""
    W_ = 32
    cam = scenegen.camera_look_at((0, 0, 10), (0, 0, 0), (0, 1, 0), W_, W_)
    th_front = math.log(0.9 / 0.1)
    s4 = 0.634  # alpha of the fourth about 0.9 at the centre with o about 0.9999

    def mk(th):
        front = [dict(mean=(0, 0, 0.5 - 0.5 * k), log_scale=(math.log(6.0),) * 3, logit=th_front,
                      rgb=(0.6, 0.6, 0.6)) for k in range(3)]
        return front + [dict(mean=(0, 0, -2.0), log_scale=(math.log(s4),) * 3, logit=th, rgb=(0.6, 0.6, 0.6))]

    def expected(t, F):
        T = np.ones((W_, W_))
        for i in range(3):
            T = T * (1.0 - np.minimum(0.99, _alpha64(t, i, cam, (W_, W_))))
        a4 = np.minimum(0.99, _alpha64(t, 3, cam, (W_, W_)))
        near = a4 > 0.5  # the fourth passes the skip test far from its threshold
        counts = F.pixel_counts()
        assert np.all(counts[near] >= 3)
        stop64 = T * (1.0 - a4) < 1e-4
        stop32 = counts == 3
        assert not np.any(stop64[~near])
        return {"stop_flip64": int((stop32 != stop64)[near].sum())}

    # the logit where T (1 - alpha_4) = 1e-4 at the central pixels in FP64
    t0 = single_splat_tree(mk(0.0))
    T = 1.0
    for i in range(3):
        T *= 1.0 - min(0.99, _alpha64(t0, i, cam, (W_, W_))[16, 16])
    th_star = _logit_at(1.0 - 1e-4 / T, t0, 3, cam, (W_, W_), 16, 16)
    assert 7.0 < th_star < 11.0
    thetas = _fine_thetas(th_star - 100 * 4.8e-7, 200)
    got, want = _flip_sweep(mk, thetas, cam, expected)
    assert got["stop_flip64"] == want["stop_flip64"]
    assert got["stop_flip64"] > 0


def test_flip_counts_small_on_a_scene(tiny_tree, tiny_oracle):
    """On the tiny scene the FP64 evaluation disagrees with the FP32 mirror on a
    vanishing fraction of the decisions (the log exists to show exactly this)."""
    from scenegen import configs
    cam = configs.tiny_camera()
    ids, _ = tiny_oracle.select(cam, 1.0)
    F = oracle.OracleFrame(tiny_tree, ids, cam)
    info = F.info()
    total = info["n_contrib"]
    assert total > 100000
    for k in ("skip_flip64", "stop_flip64", "clamp_flip64"):
        assert 0 <= info[k] <= 1e-4 * total, (k, info[k], total)

"""Pins of the closure oracle (CPU, no GPU).

The oracle's pole-crossing padding is checked against analytic fields written
in the extended coordinates; the convolution against scipy's correlation; the
backward pass against central finite differences of the forward pass; Adam's
first step against its closed form; the box filter against conservation.
"""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import closure_oracle as CO


def _grid(H, W):
    th = (np.arange(H) + 0.5) * np.pi / H
    ph = (np.arange(W) + 0.5) * 2 * np.pi / W
    return th, ph


def _scalar(th, ph):
    # a smooth function of the Cartesian position (x + 2y + 3z + xz)
    x, y, z = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
    return x + 2 * y + 3 * z + x * z


def _vector(th, ph):
    # solid-body rotation about the x axis, u = x_hat cross r = (0, -z, y),
    # projected on e_theta = (cos th cos ph, cos th sin ph, -sin th) and
    # e_phi = (-sin ph, cos ph, 0)
    y, z = np.sin(th) * np.sin(ph), np.cos(th)
    ut = -z * np.cos(th) * np.sin(ph) - y * np.sin(th)
    up = -z * np.cos(ph)
    return ut, up


@pytest.mark.parametrize("H,W", [(6, 8), (9, 12), (2, 4)])
def test_every_cell_is_read_nine_times(H, W):
    nbr, cross = CO.neighbours(H, W)
    counts = np.bincount(nbr.reshape(-1), minlength=H * W)
    assert np.all(counts == 9)
    # exactly the first and last rows read across a pole, through their 3 outer taps
    assert cross[0, :, :3].all() and cross[-1, :, 6:].all()
    assert cross.sum() == 2 * 3 * W
    assert np.all(nbr[0, :, 1] == (np.arange(W) + W // 2) % W)          # tap (-1, 0)


@pytest.mark.parametrize("H,W", [(8, 16), (5, 10)])
def test_padding_equals_the_field_in_extended_coordinates(H, W):
    # Tap (dy, dx) of cell (r, c) lies at theta = (r + dy + 1/2) dth, phi = (c +
    # dx + 1/2) dph in the extended coordinates, also beyond a pole; a smooth
    # scalar written in those coordinates must equal the gathered value, and so
    # must the orthonormal components of a smooth vector field.
    th, ph = _grid(H, W)
    nbr, cross = CO.neighbours(H, W)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ut, up = _vector(TH, PH)
    x = np.stack([_scalar(TH, PH), ut, up], axis=-1)[None]
    g = CO.gather(x, nbr, cross, vector_channels=(1, 2))[0]
    dth, dph = np.pi / H, 2 * np.pi / W
    for t, (dy, dx) in enumerate(CO.taps()):
        the = TH + dy * dth
        phe = PH + dx * dph
        ev = _vector(the, phe)
        np.testing.assert_allclose(g[:, :, t, 0], _scalar(the, phe), atol=1e-13)
        np.testing.assert_allclose(g[:, :, t, 1], ev[0], atol=1e-13)
        np.testing.assert_allclose(g[:, :, t, 2], ev[1], atol=1e-13)


def test_wrong_vector_sign_would_be_caught():
    # the same check with the velocity treated as a scalar fails at the poles
    H, W = 8, 16
    th, ph = _grid(H, W)
    nbr, cross = CO.neighbours(H, W)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ut, _ = _vector(TH, PH)
    g = CO.gather(ut[None, :, :, None], nbr, cross, vector_channels=())[0]
    ev = _vector(TH - np.pi / H, PH)[0]
    assert np.abs(g[0, :, 1, 0] - ev[0]).max() > 0.1


def test_conv_matches_scipy_correlation_with_periodic_phi():
    rng = np.random.default_rng(0)
    B, H, W, Cin, Cout = 2, 7, 10, 3, 4
    x = rng.normal(size=(B, H, W, Cin))
    w = rng.normal(size=(Cout, 9, Cin))
    b = rng.normal(size=Cout)
    nbr, cross = CO.neighbours(H, W)
    z = CO.conv_forward(x, w, b, nbr, cross)
    for bb in range(B):
        for co in range(Cout):
            ref = np.full((H - 2, W), b[co])
            for ci in range(Cin):
                xp = np.concatenate([x[bb, :, -1:, ci], x[bb, :, :, ci], x[bb, :, :1, ci]], axis=1)
                ref += correlate2d(xp, w[co, :, ci].reshape(3, 3), mode="valid")
            np.testing.assert_allclose(z[bb, 1:-1, :, co], ref, rtol=1e-12, atol=1e-12)


def _fd(f, a, idx, h=1e-6):
    a0 = a[idx]
    a[idx] = a0 + h
    fp = f()
    a[idx] = a0 - h
    fm = f()
    a[idx] = a0
    return (fp - fm) / (2 * h)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    B, H, W, Cin, Cout = 2, 4, 6, 3, 2
    x = rng.normal(size=(B, H, W, Cin))
    w = rng.normal(size=(Cout, 9, Cin))
    b = rng.normal(size=Cout)
    dz = rng.normal(size=(B, H, W, Cout))
    nbr, cross = CO.neighbours(H, W)
    vc = (1, 2)
    f = lambda: float((dz * CO.conv_forward(x, w, b, nbr, cross, vc)).sum())
    dx, dw, db = CO.conv_backward(x, w, dz, nbr, cross, vc)
    for idx in [(0, 0, 0, 1), (1, 3, 5, 2), (0, 0, 3, 0), (1, 2, 2, 1)]:
        assert abs(_fd(f, x, idx) - dx[idx]) < 1e-7 * (1 + abs(dx[idx]))
    for idx in [(0, 0, 0), (1, 4, 2), (0, 8, 1)]:
        assert abs(_fd(f, w, idx) - dw[idx]) < 1e-7 * (1 + abs(dw[idx]))
    for i in range(Cout):
        assert abs(_fd(f, b, (i,)) - db[i]) < 1e-7 * (1 + abs(db[i]))


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    B, H, W = 2, 4, 8
    params = CO.init_params(rng, hidden=5)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in params]   # nonzero biases
    x = rng.normal(size=(B, H, W, 3))
    tgt = rng.normal(size=(B, H, W, 3))
    nbr, cross = CO.neighbours(H, W)

    def loss():
        z, _ = CO.net_forward(params, x, nbr, cross)
        return CO.loss_and_grad(z, tgt, H)[0]

    z, cache = CO.net_forward(params, x, nbr, cross)
    _, dz = CO.loss_and_grad(z, tgt, H)
    grads = CO.net_backward(params, cache, dz, nbr, cross)
    for li, idx in [(0, (1, 4, 2)), (1, (3,)), (2, (2, 7, 4)), (3, (0,)), (4, (1, 0, 3)), (5, (2,))]:
        g_fd = _fd(loss, params[li], idx)
        assert abs(g_fd - grads[li][idx]) < 1e-6 * (1 + abs(g_fd)), (li, idx)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -2e-3, 0.5])
    p, m, v = CO.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_box_filter_conserves_mass_and_momentum():
    rng = np.random.default_rng(3)
    H, W, f = 16, 32, 4
    rho = 1 + 0.1 * rng.random((H, W))
    ut, up = rng.normal(size=(H, W)), rng.normal(size=(H, W))
    rc, uc, vc = CO.box_filter(rho, ut, up, f)
    wf = CO.row_weights(H)[:, None]
    wc = wf.reshape(H // f, f).sum(axis=1)[:, None] * f
    assert np.isclose((wf * rho).sum(), (wc * rc).sum(), rtol=1e-13)
    assert np.isclose((wf * rho * ut).sum(), (wc * rc * uc).sum(), rtol=1e-12)
    assert np.isclose((wf * rho * up).sum(), (wc * rc * vc).sum(), rtol=1e-12)
    r1, u1, v1 = CO.box_filter(np.full((H, W), 1.3), np.full((H, W), 0.2), np.zeros((H, W)), f)
    assert np.allclose(r1, 1.3) and np.allclose(u1, 0.2) and np.allclose(v1, 0.0)

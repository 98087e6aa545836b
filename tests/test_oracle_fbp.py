"""Pins of the FBP oracle (the initial iterate of Section I) against what the
mathematics fixes: the discrete Ram-Lak kernel has the ramp |f| as its
frequency response; exact projections of a uniform disc reconstruct the
disc; back-projecting a constant gives pi; hand-placed protons land in the
bins worked out by hand; straight protons through a uniform cylinder with
exact WEPLs reconstruct the cylinder."""
import numpy as np
import pytest

from oracle import fbp
from paper_1802_01070_amd import synth


def test_ramlak_response_is_the_ramp():
    # dt sum_m h(m) e^{-i w m} = |w| / (2 pi dt) = |f| for f = w / (2 pi dt),
    # from the Fourier series sum_{odd m>0} cos(m w) / m^2 = pi/4 (pi/2 - |w|)
    n_t, dt = 4097, 0.5
    c = n_t // 2
    p = np.zeros((1, 1, n_t))
    p[0, 0, c] = 1.0
    q = fbp.filter_rows(p, dt)[0, 0]
    k = np.arange(n_t) - c
    f = np.linspace(0.0, 1.0 / (2 * dt), 41)
    resp = np.array([np.sum(q * np.exp(-2j * np.pi * fi * k * dt)) for fi in f])
    assert np.max(np.abs(resp.imag)) < 1e-9            # even kernel
    # the kernel is cut at |m| <= 2048: tail <= 2 / (pi^2 dt) * 1 / (2 * 2047)
    assert np.max(np.abs(resp.real - f)) < 1e-3
    # zero frequency: the taps sum to ~0 (no DC), the centre tap is 1 / (4 dt)
    assert abs(q[c] - 1.0 / (4 * dt)) < 1e-15
    assert q[c + 2] == 0.0 and q[c - 4] == 0.0


def test_disc_projections_reconstruct_the_disc():
    R, mu, dt, n_t, n_ang = 40.0, 1.2, 0.5, 256, 360
    grid = synth.Grid(128, 128, 1)
    t0 = -n_t * dt / 2
    tc = t0 + (np.arange(n_t) + 0.5) * dt
    row = 2 * mu * np.sqrt(np.clip(R * R - tc * tc, 0.0, None))
    p = np.broadcast_to(row, (1, n_ang, n_t)).copy()
    x = fbp.backproject(grid, fbp.filter_rows(p, dt), n_ang, t0, dt)
    ix, iy = np.arange(grid.nvox) % grid.nx, np.arange(grid.nvox) // grid.nx
    r = np.hypot(grid.origin[0] + ix + 0.5, grid.origin[1] + iy + 0.5)
    inside, outside = r < 0.8 * R, (r > 1.2 * R) & (r < 60.0)
    assert abs(x[inside].mean() - mu) < 0.005 * mu
    assert np.max(np.abs(x[inside] - mu)) < 0.02 * mu
    assert np.max(np.abs(x[outside])) < 0.03 * mu


def test_backprojection_of_a_constant_is_pi():
    grid = synth.Grid(16, 16, 2)
    n_t, dt, n_ang = 40, 1.0, 12
    t0 = -20.0
    q = np.ones((2, n_ang, n_t))
    x = fbp.backproject(grid, q, n_ang, t0, dt)
    # every voxel centre of the 16 mm grid is within 11.4 mm of the axis, so
    # all its samples fall between bin centres -19.5 .. 19.5
    np.testing.assert_allclose(x, np.pi, rtol=1e-14)
    # a single bin: the back-projection of one angle is the hat of width 2 dt
    q = np.zeros((2, n_ang, n_t))
    q[1, 0, 20] = 1.0           # angle 0 (t = y), centre t = 0.5
    x = fbp.backproject(grid, q, n_ang, t0, dt).reshape(2, 16, 16)
    yc = -8 + np.arange(16) + 0.5
    hat = np.clip(1.0 - np.abs(yc - 0.5) / dt, 0.0, None) * np.pi / n_ang
    np.testing.assert_allclose(x[1], np.repeat(hat[:, None], 16, axis=1), atol=1e-15)
    assert not x[0].any()


def test_binning_by_hand():
    grid = synth.Grid(4, 4, 2)                       # origin (-2, -2, -1)
    mlp = synth.MLPModel(u_in=-10.0, u_out=10.0)     # chord centre: mean of entry and exit
    n_ang, n_t, t0, dt = 4, 4, -2.0, 1.0
    q = np.pi / 2
    # (t_in, v_in, th, ph, t_out, v_out, th, ph, gantry), b
    rays = [((0.25, 0.5, 0, 0, 0.25, 0.5, 0, 0, q + 0.1), 3.0),          # bin (1, 1, 2)
            ((0.75, 0.25, 0, 0, -0.25, 0.75, 0, 0, q - 0.2), 5.0),       # t_c 0.25, v_c 0.5: same bin
            ((-1.5, -0.9, 0, 0, 0.5, 0.7, 0, 0, 2 * np.pi - 0.1), 7.0),  # t_c -0.5, v_c -0.1: (0, 0, 1)
            ((1.9, 0.1, 0, 0, 1.9, 0.1, 0, 0, 3 * q + 0.7), 2.0),        # angle 3.45 -> bin 3: (1, 3, 3)
            ((2.5, 0.1, 0, 0, 2.5, 0.1, 0, 0, 0.0), 1.0),                # t_c beyond the bins: dropped
            ((0.0, 1.5, 0, 0, 0.0, 0.9, 0, 0, 0.0), 1.0),                # v_c 1.2: above the grid, dropped
            ((0.0, 0.5, 0, 0, 0.0, 0.5, 0, 0, 0.0), np.nan),             # non-finite b: dropped
            ((0.0, 0.5, 0, 0, 0.0, 0.5, 0, 0, np.inf), 1.0),             # non-finite angle: dropped
            ((0.0, 0.5, 0, 0, 0.0, 0.5, 0, 0, 0.0), 2.0 ** 20),          # not a WEPL: dropped
            ((-2.0, -1.0, 0, 0, -2.0, -1.0, 0, 0, -0.3), 4.0)]           # lower edges, angle -0.3 -> bin 0
    pr = synth.make_rays(grid, mlp, [r for r, _ in rays])
    b = np.array([v for _, v in rays], dtype=np.float32)
    p, c = fbp.sinogram(grid, mlp, pr, b, n_ang, n_t, t0, dt)
    ep, ec = np.zeros((2, 4, 4)), np.zeros((2, 4, 4), dtype=np.int64)
    ep[1, 1, 2], ec[1, 1, 2] = 4.0, 2
    ep[0, 0, 1], ec[0, 0, 1] = 7.0, 1
    ep[1, 3, 3], ec[1, 3, 3] = 2.0, 1
    ep[0, 0, 0], ec[0, 0, 0] = 4.0, 1
    np.testing.assert_array_equal(c, ec)
    np.testing.assert_allclose(p, ep, rtol=1e-15)


def test_straight_protons_through_a_cylinder():
    # parallel straight protons (t_in = t_out, zero slopes) at 180 exact bin
    # angles; b = mu * exact chord through the cylinder of radius R
    R, mu = 30.0, 1.0
    grid = synth.Grid(96, 96, 2)
    mlp = synth.MLPModel(u_in=-48.0, u_out=48.0)
    n_ang, n_t, t0, dt = 180, 96, -48.0, 1.0
    rng = np.random.default_rng(5)
    per = 3000
    t = rng.uniform(-48.0, 48.0, n_ang * per)
    v = rng.uniform(-1.0, 1.0, n_ang * per)
    phi = np.repeat(2 * np.pi * np.arange(n_ang) / n_ang, per)
    z = np.zeros_like(t)
    pr = {k: a.astype(np.float32) for k, a in dict(t_in=t, v_in=v, th_in=z, ph_in=z, t_out=t, v_out=v,
                                                    th_out=z, ph_out=z, gantry=phi).items()}
    tt = pr["t_in"].astype(np.float64)
    b = (mu * 2 * np.sqrt(np.clip(R * R - tt * tt, 0.0, None))).astype(np.float32)
    x = fbp.fbp(grid, mlp, pr, b, n_ang, n_t, t0, dt).reshape(2, 96, 96)
    ix = np.arange(96)
    r = np.hypot(-48 + ix[None, :] + 0.5, -48 + ix[:, None] + 0.5)
    for s in range(2):
        inside = x[s][r < 0.8 * R]
        assert abs(inside.mean() - mu) < 0.01 * mu
        assert np.max(np.abs(inside - mu)) < 0.05 * mu
        assert np.max(np.abs(x[s][(r > 1.2 * R) & (r < 45)])) < 0.05 * mu


@pytest.mark.parametrize("plant", ["sign", "scale"])
def test_planted_filter_mistakes_fail_the_disc_pin(plant, monkeypatch):
    # a plausible mistake in the kernel (wrong sign of the odd taps, or a
    # missing dt) must break the disc reconstruction
    real = fbp.ramlak

    def wrong(n_t, dt):
        h = real(n_t, dt)
        if plant == "sign":
            m = np.arange(-(n_t - 1), n_t)
            h[m % 2 != 0] *= -1
        else:
            h *= dt
        return h

    monkeypatch.setattr(fbp, "ramlak", wrong)
    R, mu, dt, n_t, n_ang = 40.0, 1.2, 0.5, 256, 90
    grid = synth.Grid(64, 64, 1, pitch=(2.0, 2.0, 1.0))
    t0 = -n_t * dt / 2
    tc = t0 + (np.arange(n_t) + 0.5) * dt
    p = np.broadcast_to(2 * mu * np.sqrt(np.clip(R * R - tc * tc, 0.0, None)), (1, n_ang, n_t)).copy()
    x = fbp.backproject(grid, fbp.filter_rows(p, dt), n_ang, t0, dt)
    ix, iy = np.arange(grid.nvox) % 64, np.arange(grid.nvox) // 64
    r = np.hypot(-64 + 2 * ix + 1.0, -64 + 2 * iy + 1.0)
    assert abs(x[r < 0.8 * R].mean() - mu) > 0.05 * mu

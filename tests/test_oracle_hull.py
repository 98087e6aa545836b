"""Pins of the oracle's per-proton paths through an object hull (the MLP
evaluated between the points where the tracks enter and leave the object,
Section I; straight tracks outside): the hull crossings lie on the hull circle
and on the measured tracks, a hull that contains the tracker span gives the
tracker-to-tracker path exactly, a missed hull gives one straight segment,
consistent straight input stays straight, and the MLP part is the MLP of the
same proton with its tracker planes moved to the hull crossings."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1802_01070_amd import synth


@pytest.fixture(autouse=True)
def _hull_off():
    oracle.build(force=False)
    oracle.set_hull(None)
    yield
    oracle.set_hull(None)


def beam_to_lab(u, t, v, phi):
    return np.array([u * np.cos(phi) - t * np.sin(phi), u * np.sin(phi) + t * np.cos(phi), v])


def test_hull_crossings_lie_on_the_circle_and_the_tracks():
    sc = synth.make_scan(synth.WORKLOADS[1], m=400)
    m = sc.mlp
    R = 24.0
    oracle.set_hull(R, 0.5, -0.25)
    n_hit = 0
    for i in range(sc.m):
        P = oracle.path(m, sc.protons, i)
        f = {k: float(v[i]) for k, v in sc.protons.items()}
        if len(P) == 2:                       # missed: the tracker points
            assert np.allclose(P[0], beam_to_lab(m.u_in, f["t_in"], f["v_in"], f["gantry"]), atol=1e-12)
            assert np.allclose(P[1], beam_to_lab(m.u_out, f["t_out"], f["v_out"], f["gantry"]), atol=1e-12)
            continue
        n_hit += 1
        # entry crossing first: beam-frame depths increase along the polyline
        depth = P[:, 0] * np.cos(f["gantry"]) + P[:, 1] * np.sin(f["gantry"])
        assert np.all(np.diff(depth) > 0)
        # first and last vertices are the tracker points (hull inside the planes here)
        assert np.allclose(P[0], beam_to_lab(m.u_in, f["t_in"], f["v_in"], f["gantry"]), atol=1e-12)
        assert np.allclose(P[-1], beam_to_lab(m.u_out, f["t_out"], f["v_out"], f["gantry"]), atol=1e-12)
        for h, (t0, th, v0, ph, u0) in ((P[1], (f["t_in"], f["th_in"], f["v_in"], f["ph_in"], m.u_in)),
                                        (P[-2], (f["t_out"], f["th_out"], f["v_out"], f["ph_out"], m.u_out))):
            assert np.hypot(h[0] - 0.5, h[1] + 0.25) == pytest.approx(R, abs=1e-9)
            u = h[0] * np.cos(f["gantry"]) + h[1] * np.sin(f["gantry"])       # beam-frame depth of the point
            assert np.allclose(h, beam_to_lab(u, t0 + th * (u - u0), v0 + ph * (u - u0), f["gantry"]), atol=1e-9)
    assert n_hit > sc.m // 2


def test_hull_containing_the_trackers_is_the_tracker_path():
    sc = synth.make_scan(synth.WORKLOADS[1], m=300)
    ref_v, ref_c, ref_n = oracle.trace(sc.grid, sc.mlp, sc.protons)
    oracle.set_hull(1.0e4)
    v, c, n = oracle.trace(sc.grid, sc.mlp, sc.protons)
    assert np.array_equal(n, ref_n) and np.array_equal(v, ref_v) and np.array_equal(c, ref_c)
    for i in range(0, sc.m, 37):
        oracle.set_hull(1.0e4)
        P = oracle.path(sc.mlp, sc.protons, i)
        oracle.set_hull(None)
        assert np.array_equal(P, oracle.path(sc.mlp, sc.protons, i))


def test_mlp_part_is_the_mlp_between_the_hull_crossings():
    sc = synth.make_scan(synth.WORKLOADS[1], m=200)
    m = sc.mlp
    oracle.set_hull(22.0)
    checked = 0
    for i in range(sc.m):
        P = oracle.path(m, sc.protons, i)
        if len(P) == 2:
            continue
        f = {k: float(v[i]) for k, v in sc.protons.items()}
        u_of = lambda q: q[0] * np.cos(f["gantry"]) + q[1] * np.sin(f["gantry"])
        u1, u2 = u_of(P[1]), u_of(P[-2])
        # the same proton with its trackers moved to the hull crossings
        m2 = dataclasses.replace(m, u_in=u1, u_out=u2)
        one = {k: v[i:i + 1].copy() for k, v in sc.protons.items()}
        one["t_in"][0] = f["t_in"] + f["th_in"] * (u1 - m.u_in)
        one["v_in"][0] = f["v_in"] + f["ph_in"] * (u1 - m.u_in)
        one["t_out"][0] = f["t_out"] + f["th_out"] * (u2 - m.u_out)
        one["v_out"][0] = f["v_out"] + f["ph_out"] * (u2 - m.u_out)
        oracle.set_hull(None)
        inner = oracle.path(m2, one, 0)
        oracle.set_hull(22.0)
        # float32 storage of the moved states: agree to float32 resolution
        np.testing.assert_allclose(P[1:-1], inner, rtol=0, atol=2e-5)
        checked += 1
    assert checked > 50


def test_consistent_straight_tracks_stay_straight_through_the_hull():
    # a straight track (exit = entry continued, equal slopes) gives a straight
    # MLP inside the hull and straight air segments: all vertices collinear
    m = synth.MLPModel(u_in=-30.0, u_out=30.0)
    D = m.depth
    rays = [(1.5 + k, 0.25 * k - 1.0, 0.01 * k, -0.005 * k, 1.5 + k + 0.01 * k * D, 0.25 * k - 1.0 - 0.005 * k * D,
             0.01 * k, -0.005 * k, 0.3 * k) for k in range(8)]
    pr = synth.make_rays(synth.Grid(64, 64, 4), m, rays)
    oracle.set_hull(20.0)
    for i in range(len(rays)):
        P = oracle.path(m, pr, i)
        d = P[-1] - P[0]
        for q in P:
            w = q - P[0]
            assert np.linalg.norm(np.cross(w, d)) / np.linalg.norm(d) < 1e-6

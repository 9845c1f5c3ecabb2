"""Pins of the oracle's single-particle arithmetic against closed forms and invariants.

Each test fixes the oracle to something other than itself: orthogonality and
exact gyration of the Boris map (Appendix A.1), the defining implicit equation
of each rotation, the damped-oscillator recurrence of the modified Boris
scheme (Appendix A.3, Taflove form), the driven Lorentz response
(eq:lordielectric), Dirac speed renormalisation (Sec. 5) and specular
reflection (Sec. 3).
"""
import math

import numpy as np
import pytest

QE = 1.602176634e-19
ME = 9.1093837015e-31


def eps_matrix(b):
    # eps(b) u = u x b, the matrix printed below eq:borisrotsol
    return np.array([[0.0, b[2], -b[1]], [-b[2], 0.0, b[0]], [b[1], -b[0], 0.0]])


def test_eps_matrix_is_cross_product():
    rng = np.random.default_rng(0)
    for _ in range(10):
        b, u = rng.normal(size=3), rng.normal(size=3)
        assert np.allclose(eps_matrix(b) @ u, np.cross(u, b), rtol=0, atol=1e-15)


def test_boris_matrix_solves_implicit_rotation(oracle):
    # eq:borisrot: v+ - v- = (v+ + v-) x b  <=>  (I - eps(b)) v+ = (I + eps(b)) v-
    rng = np.random.default_rng(1)
    for _ in range(50):
        b = rng.normal(size=3) * rng.choice([1e-3, 0.3, 3.0])
        R = oracle.boris_matrix(b)
        vm = rng.normal(size=3)
        vp_exact = np.linalg.solve(np.eye(3) - eps_matrix(b), (np.eye(3) + eps_matrix(b)) @ vm)
        assert np.allclose(R @ vm, vp_exact, rtol=1e-14, atol=1e-14)
        assert np.allclose(R @ R.T, np.eye(3), atol=2e-15)
        assert abs(np.linalg.det(R) - 1.0) < 2e-15


def test_boris_gyration_speed_phase_radius(oracle):
    # P1: pure B: |v| conserved; phase per step 2 atan(wc dt/2); orbit radius r_L sqrt(1+(wc dt/2)^2)
    qm = -QE / ME
    Bz = 10.0
    wc = abs(qm) * Bz
    dt = 0.3 / wc
    v = np.array([1.0e6, 0.0, 2.0e5])
    x = np.zeros(3)
    xs, vs = [x.copy()], [v.copy()]
    for _ in range(2000):
        v = oracle.push_free(qm, dt, [0, 0, 0], [0, 0, Bz], v)
        x = x + dt * v
        xs.append(x.copy()); vs.append(v.copy())
    vs = np.array(vs); xs = np.array(xs)
    speed = np.linalg.norm(vs, axis=1)
    assert np.max(np.abs(speed / speed[0] - 1.0)) < 2000 * 1e-15 + 1e-14
    vperp = vs[:, 0] + 1j * vs[:, 1]
    dphi = np.angle(vperp[1:] / vperp[:-1])
    expect = 2.0 * math.atan(wc * dt / 2.0)
    assert np.max(np.abs(np.abs(dphi) - expect)) < 1e-13
    # the positions lie on a circle; fit its centre from three points and compare radii
    vp = math.hypot(1.0e6, 0.0)
    r_expect = vp / wc * math.sqrt(1.0 + (wc * dt / 2.0) ** 2)
    p = xs[:, :2]
    a, b, c = p[10], p[400], p[1300]
    A = np.array([[b[0] - a[0], b[1] - a[1]], [c[0] - a[0], c[1] - a[1]]]) * 2.0
    rhs = np.array([b @ b - a @ a, c @ c - a @ a])
    centre = np.linalg.solve(A, rhs)
    radii = np.linalg.norm(p - centre, axis=1)
    assert np.max(np.abs(radii / r_expect - 1.0)) < 1e-9
    # v_z untouched
    assert np.all(vs[:, 2] == 2.0e5)


def test_boris_exb_drift_is_fixed_point(oracle):
    qm = -QE / ME
    E = np.array([3.0e7, -1.0e7, 0.0])
    B = np.array([0.0, 0.0, 5.0])
    vd = np.cross(E, B) / (B @ B)
    v = vd.copy()
    dt = 1e-15
    for _ in range(100):
        v = oracle.push_free(qm, dt, E, B, v)
    assert np.allclose(v, vd, rtol=1e-13, atol=1e-9)


def test_boris_electric_kick(oracle):
    # B = 0: v_{n+1/2} = v_{n-1/2} + dt (q/m) E exactly (two half kicks)
    qm = -QE / ME
    v = oracle.push_free(qm, 1e-17, [1e9, -2e9, 3e8], [0, 0, 0], [1.0, 2.0, 3.0])
    assert np.allclose(v, np.array([1.0, 2.0, 3.0]) + 1e-17 * qm * np.array([1e9, -2e9, 3e8]), rtol=1e-15)


def test_gyro_matrix_reductions_and_defining_equation(oracle):
    rng = np.random.default_rng(2)
    for _ in range(30):
        b = rng.normal(size=3) * 0.4
        g = rng.uniform(0.0, 0.3, size=3)
        R = oracle.gyro_matrix(b, g)
        vm = rng.normal(size=3)
        vp = R @ vm
        # (v+ - v-) = (eps(b) - G)(v+ + v-), G = diag(g): the rotation equation with dt/2 absorbed
        lhs = vp - vm
        rhs = (eps_matrix(b) - np.diag(g)) @ (vp + vm)
        assert np.allclose(lhs, rhs, rtol=1e-13, atol=1e-14)
        # gamma = 0 reduces to eq:borisrotsol
        assert np.allclose(oracle.gyro_matrix(b, [0, 0, 0]), oracle.boris_matrix(b), atol=1e-15)
        # B = 0 reduces to eq:modborisrotsol, diag((1-g)/(1+g))
        assert np.allclose(oracle.gyro_matrix([0, 0, 0], g), np.diag((1 - g) / (1 + g)), atol=1e-16)


def test_printed_gyro_numerator_is_not_a_rotation():
    # The closed form printed for the gyrotropic rotation does not reduce to a rotation at gamma = 0
    # (it does not preserve |v|), which is why the oracle solves L- v+ = L+ v- directly.
    b = np.array([0.3, -0.2, 0.5])
    g = np.zeros(3)
    G = np.diag(g)
    detIG = np.linalg.det(np.eye(3) + G)
    num = (np.eye(3) - G) @ np.linalg.inv(np.eye(3) + G) * detIG + eps_matrix((np.eye(3) + G) @ b) + np.outer(b, b)
    det_lm = detIG + b @ ((np.eye(3) + G) @ b)
    R_printed = num / det_lm
    v = np.array([1.0, 0.5, -0.3])
    assert abs(np.linalg.norm(R_printed @ v) / np.linalg.norm(v) - 1.0) > 1e-3


def test_bound_push_taflove_recurrence(oracle):
    # Appendix A.3 (read with dt^2): x_{n+1} - 2x_n + x_{n-1} = dt^2 (q/m E - w2 x_n) - (g dt/2)(x_{n+1} - x_{n-1})
    qm = -QE / ME
    w2 = np.array([6.0e15, 5.0e15, 4.0e15]) ** 2
    gam = np.array([1.5e14, 3.0e14, 0.0])
    dt = 2.0e-18
    xi = np.array([1e-11, -5e-12, 2e-12])
    v = np.zeros(3)
    xs = [xi.copy()]
    rng = np.random.default_rng(3)
    Es = rng.normal(size=(400, 3)) * 1e8
    for n in range(400):
        v = oracle.push_bound(qm, dt, w2, gam, 0.0, Es[n], [0, 0, 0], xi, v)
        xi = xi + dt * v
        xs.append(xi.copy())
    xs = np.array(xs)
    for n in range(1, 400):
        lhs = xs[n + 1] - 2 * xs[n] + xs[n - 1] + (gam * dt / 2.0) * (xs[n + 1] - xs[n - 1])
        rhs = dt * dt * (qm * Es[n] - w2 * xs[n])
        scale = np.abs(xs[n]) + np.abs(xs[n + 1]) + 1e-30
        assert np.all(np.abs(lhs - rhs) <= 1e-13 * scale + 1e-28)


def test_bound_push_free_oscillation_roots(oracle):
    # P3: E = 0: characteristic roots of (1+g) z^2 - (2 - w^2 dt^2) z + (1-g) = 0
    w0 = 6.077e15
    gamma = 1.519e14
    dt = 2.24e-18
    g = gamma * dt / 2.0
    z = np.roots([1 + g, -(2 - (w0 * dt) ** 2), 1 - g])
    z = z[np.argmax(z.imag)]
    assert abs(abs(z) ** 2 - (1 - g) / (1 + g)) < 1e-15
    xi = np.array([1e-11, 0.0, 0.0])
    v = np.zeros(3)
    xs = [xi[0]]
    for _ in range(3000):
        v = oracle.push_bound(-QE / ME, dt, [w0 * w0] * 3, [gamma] * 3, 0.0, [0, 0, 0], [0, 0, 0], xi, v)
        xi = xi + dt * v
        xs.append(xi[0])
    xs = np.array(xs)
    # the trajectory is A z^n + conj: x_{n+1} = 2 Re(z) x_n - |z|^2 x_{n-1}
    pred = 2 * z.real * xs[1:-1] - abs(z) ** 2 * xs[:-2]
    assert np.max(np.abs(pred - xs[2:])) < 1e-12 * np.max(np.abs(xs))
    # damped frequency tends to sqrt(w0^2 - gamma^2/4)
    assert abs(np.angle(z) / dt / math.sqrt(w0 ** 2 - gamma ** 2 / 4) - 1.0) < 1e-3


def test_bound_push_driven_response_matches_lorentz_dielectric(oracle):
    # eq:lordielectric: steady response x = (q/m) E0 / (w0^2 - w^2 - i gamma w) for E = E0 e^{-i w t}
    qm = -QE / ME
    w0, gamma = 6.077e15, 1.519e14
    dt = 2.24e-18
    E0 = 1e8
    for w in (0.5 * w0, 0.9 * w0, 1.3 * w0):
        xi = np.zeros(3)
        v = np.zeros(3)
        n_steps = 60000
        xs = np.zeros(n_steps)
        for n in range(n_steps):
            E = E0 * math.cos(w * n * dt)
            v = oracle.push_bound(qm, dt, [w0 * w0] * 3, [gamma] * 3, 0.0, [E, 0, 0], [0, 0, 0], xi, v)
            xi = xi + dt * v
            xs[n] = xi[0]  # x_{n+1}
        t = (np.arange(n_steps) + 1) * dt
        sel = slice(n_steps // 2, None)  # transients decayed (gamma t >> 1)
        M = np.stack([np.cos(w * t[sel]), np.sin(w * t[sel])], axis=1)
        (a, b), *_ = np.linalg.lstsq(M, xs[sel], rcond=None)
        measured = a + 1j * b  # x = Re(measured e^{-i w t})
        chi = qm * E0 / (w0 ** 2 - w ** 2 - 1j * gamma * w)
        assert abs(measured / chi - 1.0) < 1e-3, (w, measured, chi)


def test_dirac_speed_and_sheet(oracle):
    rng = np.random.default_rng(4)
    vf = 1e6
    md = oracle.dirac_mass(0.2 * QE, vf)
    qm = -QE / md
    dt = 1.12e-18
    ulp = np.spacing(vf)
    for _ in range(200):
        v0 = rng.normal(size=3)
        v0[1] = 0.0
        v0 *= vf / np.linalg.norm(v0)
        v = oracle.push_dirac(qm, dt, vf, 1, rng.normal(size=3) * 1e9, rng.normal(size=3) * 10, v0)
        assert v[1] == 0.0
        assert abs(np.linalg.norm(v) - vf) <= 2 * ulp


def test_dirac_zero_intermediate_keeps_direction(oracle):
    # q/m = 1, dt = 2 and E = -v/2 make both half kicks exactly -v/2, so v' = 0 exactly
    vf = 1e6
    v0 = np.array([0.0, 0.0, vf])
    v = oracle.push_dirac(1.0, 2.0, vf, 1, -v0 / 2, [0, 0, 0], v0)
    assert np.array_equal(v, v0)


def test_dirac_cyclotron_rotation(oracle):
    # B along the sheet normal, E = 0: |v| = v_F and the angle advances 2 atan(b) per step, b = dt q B/(2 m_d)
    vf = 1e6
    md = oracle.dirac_mass(0.2 * QE, vf)
    qm = -QE / md
    dt = 1e-16
    By = 3.0
    v = np.array([vf, 0.0, 0.0])
    ang = []
    for _ in range(50):
        v_new = oracle.push_dirac(qm, dt, vf, 1, [0, 0, 0], [0, By, 0], v)
        ang.append(np.angle((v_new[2] + 1j * v_new[0]) / (v[2] + 1j * v[0])))
        v = v_new
    expect = 2 * math.atan(abs(qm) * By * dt / 2)
    assert np.max(np.abs(np.abs(ang) - expect)) < 1e-12


def test_dirac_mass_and_density():
    from oracle import oracle as O
    md = O.dirac_mass(0.2 * QE, 1e6)
    assert abs(md / 1.602176634e-32 - 1.0) < 1e-12
    assert abs(md / ME - 0.017588) < 1e-5
    n2d = O.dirac_density2d(0.2 * QE, 1e6)  # m^-2
    assert abs(n2d * 1e-4 / 2.94e12 - 1.0) < 2e-3


def _ball_species(O, center, radius):
    return O.make_species({"kind": "free", "q": -QE, "m": ME, "reflect": True,
                           "region": {"kind": "ball", "center": center, "radius": radius}}, 2)


def test_reflection_ball(oracle):
    import ctypes as C
    rng = np.random.default_rng(5)
    sp = _ball_species(oracle, [10.0, 12.0, 0.0], 5.0)
    L = oracle.lib()
    for _ in range(200):
        ang = rng.uniform(0, 2 * np.pi)
        r = 5.0 + rng.uniform(1e-6, 0.01)
        X = np.array([10.0 + r * np.cos(ang), 12.0 + r * np.sin(ang), 0.0])
        v = rng.normal(size=3) * 1e6
        X2, v2 = X.copy(), v.copy()
        hit = L.or_reflect(C.byref(sp), 2, X2.ctypes.data_as(C.POINTER(C.c_double)),
                           v2.ctypes.data_as(C.POINTER(C.c_double)))
        assert hit == 1
        rhat = np.array([np.cos(ang), np.sin(ang), 0.0])
        r2 = np.linalg.norm(X2[:2] - [10.0, 12.0])
        assert abs(r2 - (10.0 - r)) < 1e-12  # mirrored radius 2R - r
        assert r2 <= 5.0
        assert abs(np.linalg.norm(v2) - np.linalg.norm(v)) < 1e-15 * np.linalg.norm(v) * 4
        assert abs(v2 @ rhat + v @ rhat) < 1e-14 * np.linalg.norm(v)  # normal component flips
        t = v - (v @ rhat) * rhat
        t2 = v2 - (v2 @ rhat) * rhat
        assert np.allclose(t, t2, rtol=0, atol=1e-14 * np.linalg.norm(v))
        assert v2[2] == v[2]
    # inside: untouched
    X = np.array([11.0, 12.5, 0.0]); v = np.array([1.0, 2.0, 3.0])
    assert L.or_reflect(C.byref(sp), 2, X.ctypes.data_as(C.POINTER(C.c_double)),
                        v.ctypes.data_as(C.POINTER(C.c_double))) == 0


def test_reflection_box(oracle):
    import ctypes as C
    sp = oracle.make_species({"kind": "free", "q": -QE, "m": ME, "reflect": True,
                              "region": {"kind": "box", "lo": [2.0, 3.0, 0], "hi": [8.0, 9.0, 1]}}, 2)
    X = np.array([8.25, 2.5, 0.0]); v = np.array([3.0, -4.0, 5.0])
    hit = oracle.lib().or_reflect(C.byref(sp), 2, X.ctypes.data_as(C.POINTER(C.c_double)),
                                  v.ctypes.data_as(C.POINTER(C.c_double)))
    assert hit == 1
    assert np.allclose(X, [7.75, 3.5, 0.0]) and np.allclose(v, [-3.0, 4.0, 5.0])

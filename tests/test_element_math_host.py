"""The kernels' element math (csrc/projections.h, compiled for the host) against the oracle's
projections: per-triangle strain + area and per-hinge bending residual contributions, in
FP64 and FP32, from the rest shape to strongly distorted triangles."""
import ctypes
import os

import numpy as np
import pytest

import npfem_inputs as I
import oracle as O

LIB = os.path.join(os.path.dirname(__file__), "..", "paper_1911_03062_amd", "libnpfem_elemcheck.so")
dp = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnpfem_elemcheck.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    L.npfem_check_triangle.argtypes = [dp, dp] + [ctypes.c_double] * 5 + [dp, ctypes.c_int]
    L.npfem_check_hinge.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int]
    return L


def _ptr(a):
    return a.ctypes.data_as(dp)


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
@pytest.mark.parametrize("amp", [0.0, 0.01, 0.05])
def test_triangle_residuals_match_oracle(lib, kind, amp):
    x, t, m = I.cell_type_inputs()[kind]
    ct = O.CellType(x, t, m, I.DT)
    xd = ct.X + amp * np.random.default_rng(int(amp * 1000) + kind).normal(size=ct.X.shape)
    F = O.deformation_gradients(xd[None], ct)
    ps, pa = O.triangle_projections(F, ct)
    M = ct.area[None, :, None, None] * (ct.w_s * (F - ps) + ct.w_a * (F - pa))
    ref = np.einsum("nmdk,mjk->mjd", M, ct.G)
    # FP32 noise floor: w_a A |g| times FP32 strain resolution (~1e-7 relative on positions)
    floor32 = 1e-6 * np.max(ct.w_a * ct.area * np.abs(ct.G).max(axis=(1, 2)))
    for prec, rtol in ((64, 1e-10), (32, 1e-5)):
        err = 0.0
        for ti in range(ct.m):
            p = np.ascontiguousarray(xd[ct.tri[ti]].ravel())
            g = np.ascontiguousarray([ct.G[ti, 1, 0], ct.G[ti, 1, 1], ct.G[ti, 2, 0], ct.G[ti, 2, 1]])
            out = np.zeros(9)
            lib.npfem_check_triangle(_ptr(p), _ptr(g), ct.area[ti], ct.w_s, ct.w_a, ct.s_min,
                                     ct.s_max, _ptr(out), prec)
            err = max(err, np.abs(out.reshape(3, 3) - ref[ti]).max())
        tol = rtol * np.abs(ref).max() + (floor32 * 100 if prec == 32 else 1e-9)
        assert err <= tol, (prec, err, tol)


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
def test_hinge_residuals_match_oracle(lib, kind):
    x, t, m = I.cell_type_inputs()[kind]
    ct = O.CellType(x, t, m, I.DT)
    xd = ct.X + 0.05 * np.random.default_rng(3).normal(size=ct.X.shape)
    u = O.bending_vectors(xd[None], ct)[0]
    W = ct.w_b * (u - O.bending_projection(u[None], ct)[0])
    ref = ct.coef[:, :, None] * W[:, None, :]
    for prec, rtol in ((64, 1e-11), (32, 1e-5)):
        err = 0.0
        for h in range(ct.e):
            p = np.ascontiguousarray(xd[ct.hinge[h]].ravel())
            a = np.ascontiguousarray(ct.coef[h])
            out = np.zeros(12)
            lib.npfem_check_hinge(_ptr(p), _ptr(a), ct.rest_norm[h], ct.w_b, _ptr(out), prec)
            err = max(err, np.abs(out.reshape(4, 3) - ref[h]).max())
        assert err <= rtol * np.abs(ref).max(), (prec, err)


def test_area_root_extreme_stretches(lib):
    """Flat triangles stretched up to 5x one way and 0.2x the other: the FP64 residual equals
    the oracle's (bracketed root), where a plain Newton from sqrt(s1/s2) diverges."""
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 0.8, 0]])
    tri = np.array([[0, 1, 2], [0, 2, 1], [0, 1, 2], [0, 1, 2]])
    G, area = O.triangle_rest_frames(X, tri[:1])
    ct = O.CellType(*I.tetrahedron(), I.RBC_MATERIAL, I.DT)
    for s1, s2 in [(5.0, 0.2), (2.2, 0.9), (1.6, 0.35), (0.5, 0.3), (3.0, 2.9)]:
        xs = X * np.array([s1, s2, 1.0])
        F = np.einsum("jd,jk->dk", xs, G[0])[None, None]
        ps, pa = O.triangle_projections(F, ct)
        M = area[0] * (ct.w_s * (F - ps) + ct.w_a * (F - pa))
        ref = np.einsum("nmdk,jk->jd", M, G[0])
        p = np.ascontiguousarray(xs.ravel())
        g = np.ascontiguousarray([G[0, 1, 0], G[0, 1, 1], G[0, 2, 0], G[0, 2, 1]])
        out = np.zeros(9)
        lib.npfem_check_triangle(_ptr(p), _ptr(g), area[0], ct.w_s, ct.w_a, ct.s_min, ct.s_max,
                                 _ptr(out), 64)
        assert np.abs(out.reshape(3, 3) - ref).max() <= 1e-9 * np.abs(ref).max(), (s1, s2)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("s", [0.6, 1.5, 2.5, 4.0])
def test_area_projection_of_isotropic_stretch_is_nearest(lib, prec, s):
    """An isotropic stretch s (sigma1 = sigma2, where the SVD basis is arbitrary and for s > 2
    two area-preserving stretches (d, 1/d) and (1/d, d) are equally near): with w_s = 0 and
    unit area the residual contributions are (F - p_a) g_j, so ||F - p_a|| recovered from
    them must equal the distance to the nearest (d, 1/d), d the minimiser of
    (t - s)^2 + (1/t - s)^2 (t = 1 for s <= 2, else the larger root of t^2 - s t + 1)."""
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 0.8, 0]])
    G, _ = O.triangle_rest_frames(X, np.array([[0, 1, 2]]))
    xs = X * s
    p = np.ascontiguousarray(xs.ravel())
    g = np.ascontiguousarray([G[0, 1, 0], G[0, 1, 1], G[0, 2, 0], G[0, 2, 1]])
    out = np.zeros(9)
    lib.npfem_check_triangle(_ptr(p), _ptr(g), 1.0, 0.0, 1.0, 1.0, 1.0, _ptr(out), prec)
    # contributions of vertices b, c are M g_b, M g_c with M = F - p_a (3 x 2)
    cb, cc = out.reshape(3, 3)[1], out.reshape(3, 3)[2]
    M = np.stack([cb, cc], axis=1) @ np.linalg.inv(np.stack([G[0, 1], G[0, 2]], axis=1))
    d = 1.0 if s <= 2.0 else 0.5 * (s + np.sqrt(s * s - 4.0))
    dist = np.hypot(s - d, s - 1.0 / d)
    tol = 1e-10 if prec == 64 else 2e-5
    assert abs(np.linalg.norm(M) - dist) <= tol * s, (s, np.linalg.norm(M), dist)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("s1", [0.5, 1.0, 2.0])
def test_projections_of_a_collinear_triangle(lib, prec, s1):
    """A triangle collapsed onto a line (F of rank one, sigma2 = 0), where the SVD's second
    left vector is any unit vector orthogonal to the first: the strain projection (polar
    factor) must have orthonormal columns, map F's right singular vector v1 to u1, and lie at
    distance sqrt((s1 - 1)^2 + 1) from F; the area projection must have singular values
    (d, 1/d) with d the largest root of t^4 - s1 t^3 - 1 and lie at distance
    sqrt((s1 - d)^2 + 1/d^2). Both projections are recovered from the residual contributions
    (F - p) g_j with one weight set to zero."""
    X = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 0.8, 0]])
    G, _ = O.triangle_rest_frames(X, np.array([[0, 1, 2]]))
    Gm = np.stack([G[0, 1], G[0, 2]], axis=1)
    # deformed positions on the x axis: F = [x_b - x_a, x_c - x_a] G has rank one
    v = np.array([0.6, 0.8])                       # unit right singular vector in the frame
    F = np.zeros((3, 2))
    F[0] = s1 * v                                  # F = s1 e_x v^T
    E = F @ np.linalg.inv(Gm.T)                    # edge vectors: F = [x_b - x_a, x_c - x_a] Gm^T
    xs = np.array([[0.2, 0.0, 0.0], [0.2, 0.0, 0.0] + E[:, 0], [0.2, 0.0, 0.0] + E[:, 1]])
    p = np.ascontiguousarray(xs.ravel())
    g = np.ascontiguousarray([G[0, 1, 0], G[0, 1, 1], G[0, 2, 0], G[0, 2, 1]])
    tol = 1e-10 if prec == 64 else 3e-5

    def proj(w_s, w_a):
        out = np.zeros(9)
        lib.npfem_check_triangle(_ptr(p), _ptr(g), 1.0, w_s, w_a, 1.0, 1.0, _ptr(out), prec)
        M = np.stack([out.reshape(3, 3)[1], out.reshape(3, 3)[2]], axis=1) @ np.linalg.inv(Gm)
        return F - M

    ps = proj(1.0, 0.0)
    assert np.abs(ps.T @ ps - np.eye(2)).max() <= tol, ps
    assert np.abs(ps @ v - np.array([1.0, 0.0, 0.0])).max() <= tol, ps @ v
    assert abs(np.linalg.norm(F - ps) - np.hypot(s1 - 1.0, 1.0)) <= tol
    r = np.roots([1.0, -s1, 0.0, 0.0, -1.0])
    d = max(x.real for x in r if abs(x.imag) < 1e-9 and x.real > 0)
    pa = proj(0.0, 1.0)
    sv = np.linalg.svd(pa, compute_uv=False)
    assert np.abs(sv - np.array([d, 1.0 / d])).max() <= tol * d, (sv, d)
    assert abs(np.linalg.norm(F - pa) - np.hypot(s1 - d, 1.0 / d)) <= tol * d


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
def test_vertex_roles_are_interchangeable(lib, kind):
    """The fused schedules may list an element's vertices in any order (chosen to spread LDS
    accesses over banks). Strain, area and bending energies do not depend on that order: a
    triangle's rest frame only fixes F up to an orthogonal factor on the right, which the
    projections carry along, and the bending stencil sums to zero, so any vertex can lead its
    difference form. All six orders of a triangle (frame rebuilt for each) and all rotations of a
    hinge give the oracle's per-vertex residuals."""
    import itertools
    x, t, m = I.cell_type_inputs()[kind]
    ct = O.CellType(x, t, m, I.DT)
    rng = np.random.default_rng(11 + kind)
    xd = ct.X * np.array([1.3, 0.8, 1.0]) + 0.05 * rng.normal(size=ct.X.shape)
    F = O.deformation_gradients(xd[None], ct)
    ps, pa = O.triangle_projections(F, ct)
    M = ct.area[None, :, None, None] * (ct.w_s * (F - ps) + ct.w_a * (F - pa))
    ref = np.einsum("nmdk,mjk->mjd", M, ct.G)
    scale = np.abs(ref).max()
    for ti in rng.choice(ct.m, 12, replace=False):
        for perm in itertools.permutations(range(3)):
            tp = ct.tri[ti][list(perm)]
            G, area = O.triangle_rest_frames(ct.X, tp[None])
            p = np.ascontiguousarray(xd[tp].ravel())
            g = np.ascontiguousarray([G[0, 1, 0], G[0, 1, 1], G[0, 2, 0], G[0, 2, 1]])
            out = np.zeros(9)
            lib.npfem_check_triangle(_ptr(p), _ptr(g), area[0], ct.w_s, ct.w_a, ct.s_min,
                                     ct.s_max, _ptr(out), 64)
            back = np.empty((3, 3))
            back[list(perm)] = out.reshape(3, 3)
            assert np.abs(back - ref[ti]).max() <= 1e-10 * scale, (ti, perm)
    u = O.bending_vectors(xd[None], ct)[0]
    W = ct.w_b * (u - O.bending_projection(u[None], ct)[0])
    href = ct.coef[:, :, None] * W[:, None, :]
    hscale = np.abs(href).max()
    for h in rng.choice(ct.e, 12, replace=False):
        for perm in itertools.permutations(range(4)):
            idx = list(perm)
            p = np.ascontiguousarray(xd[ct.hinge[h][idx]].ravel())
            a = np.ascontiguousarray(ct.coef[h][idx])
            out = np.zeros(12)
            lib.npfem_check_hinge(_ptr(p), _ptr(a), ct.rest_norm[h], ct.w_b, _ptr(out), 64)
            back = np.empty((4, 3))
            back[idx] = out.reshape(4, 3)
            assert np.abs(back - href[h]).max() <= 1e-10 * hscale, (h, perm)


def test_pbd_damping_helpers_match_oracle(lib):
    """The kernels' damping helpers (3x3 adjugate solve of I w = L, damped velocity), in a
    host build with FP64 sums, against the oracle's position-based damping."""
    lib.npfem_check_pbd.argtypes = [dp, dp, ctypes.c_int, ctypes.c_double, dp]
    rng = np.random.default_rng(44)
    for kind in (I.RBC, I.PLT):
        x0, t, m = I.cell_type_inputs()[kind]
        x = x0 + 0.1 * rng.normal(size=x0.shape) + 30.0
        v = rng.normal(size=x0.shape) + np.cross(rng.normal(size=3), x0)
        for kappa in (0.5, 0.9):
            ref = O.pbd_damp(x[None], v[None], kappa)[0]
            out = np.zeros_like(v)
            lib.npfem_check_pbd(_ptr(np.ascontiguousarray(x)), _ptr(np.ascontiguousarray(v)),
                                x.shape[0], kappa, _ptr(out))
            assert np.abs(out - ref).max() <= 1e-10 * np.abs(ref).max(), (kind, kappa)


def test_sorting_network_sorts_every_zero_one_input(lib):
    """The filter's compare-exchange network (Batcher's odd-even merge sort) on 8 and 16 keys:
    by the zero-one principle it sorts every input iff it sorts all 2^n vectors of 0s and 1s."""
    lib.npfem_check_sortnet01.argtypes = [ctypes.c_int]
    lib.npfem_check_sortnet01.restype = ctypes.c_int
    assert lib.npfem_check_sortnet01(8) == 0
    assert lib.npfem_check_sortnet01(16) == 0


def test_median_helper_matches_numpy(lib):
    """The kernels' median (8-, 16- and 32-key networks + middle selection) against numpy's
    median, bit for bit in FP64 and, on FP32-rounded inputs, in FP32; odd and even counts,
    repeated values."""
    lib.npfem_check_median.argtypes = [dp, ctypes.c_int, ctypes.c_int]
    lib.npfem_check_median.restype = ctypes.c_double
    rng = np.random.default_rng(45)
    for trial in range(1200):
        k = int(rng.integers(1, 33))
        vals = rng.normal(size=k) * 10.0 ** rng.integers(-3, 4)
        if trial % 3 == 0:
            vals = np.round(vals)                      # repeated values
        vals = np.ascontiguousarray(vals)
        assert lib.npfem_check_median(_ptr(vals), k, 64) == np.median(vals), (k, vals)
        v32 = np.ascontiguousarray(vals.astype(np.float32).astype(np.float64))
        got = np.float32(lib.npfem_check_median(_ptr(v32), k, 32))
        assert got == np.float32(np.median(v32)), (k, v32)


def test_rank_selection_median_matches_numpy(lib):
    """The wide-ring path (rank selection) against numpy's median, rings of 1 to 40 members."""
    lib.npfem_check_median_rank.argtypes = [dp, ctypes.c_int, ctypes.c_int]
    lib.npfem_check_median_rank.restype = ctypes.c_double
    rng = np.random.default_rng(48)
    for trial in range(300):
        k = int(rng.integers(1, 41))
        vals = rng.normal(size=k) * 100.0
        if trial % 2 == 0:
            vals = np.round(vals / 50.0)                # many repeated values
        vals = np.ascontiguousarray(vals)
        assert lib.npfem_check_median_rank(_ptr(vals), k, 64) == np.median(vals), (k, vals)
        v32 = np.ascontiguousarray(vals.astype(np.float32).astype(np.float64))
        got = np.float32(lib.npfem_check_median_rank(_ptr(v32), k, 32))
        assert got == np.float32(np.median(v32)), (k, v32)


def test_velocity_cap_helper_matches_oracle(lib):
    lib.npfem_check_cap.argtypes = [dp, ctypes.c_double, ctypes.c_int]
    rng = np.random.default_rng(46)
    v = rng.normal(size=(200, 3)) * 2.0
    for prec, tol in ((64, 1e-15), (32, 3e-7)):
        for vmax in (0.0, 0.5, 2.0):
            ref = O.cap_velocities(v, vmax)
            for i in range(v.shape[0]):
                w = np.ascontiguousarray(v[i].copy())
                lib.npfem_check_cap(_ptr(w), vmax, prec)
                assert np.abs(w - ref[i]).max() <= tol * (1 + np.abs(ref[i]).max()), (prec, vmax, i)


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
def test_skalak_element_matches_oracle(lib, kind):
    """The kernels' Skalak triangle (energy A W and contributions A P g_j) against the
    oracle's Skalak density and triangle scatter, in FP64 and FP32."""
    lib.npfem_check_skalak.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, dp, ctypes.c_int]
    lib.npfem_check_skalak.restype = ctypes.c_double
    x0, t, m = I.cell_type_inputs()[kind]
    ct = O.CellType(x0, t, m.with_membrane("skalak"), I.DT)
    rng = np.random.default_rng(95)
    x = x0[None] + 0.05 * rng.normal(size=(1,) + x0.shape)
    F = O.deformation_gradients(x, ct)
    W, P = O.skalak_density(F, ct)
    for tt in range(0, ct.m, 37):
        a, b, c = ct.tri[tt]
        pts = np.ascontiguousarray(x[0, [a, b, c]].reshape(-1))
        g = np.ascontiguousarray([ct.G[tt, 1, 0], ct.G[tt, 1, 1], ct.G[tt, 2, 0], ct.G[tt, 2, 1]])
        ref = np.stack([ct.area[tt] * P[0, tt] @ ct.G[tt, j] for j in range(3)])
        for prec, tol in ((64, 1e-10), (32, 2e-3)):
            out = np.zeros(9)
            E = lib.npfem_check_skalak(_ptr(pts), _ptr(g), ct.area[tt], ct.w_s, ct.w_a, _ptr(out), prec)
            scale = np.abs(ref).max() + 1e-3 * ct.w_s * ct.area[tt]
            assert np.abs(out.reshape(3, 3) - ref).max() <= tol * scale, (prec, tt)
            assert abs(E - ct.area[tt] * W[0, tt]) <= tol * (abs(ct.area[tt] * W[0, tt]) + 1e-3 * ct.w_s * ct.area[tt]), (prec, tt)

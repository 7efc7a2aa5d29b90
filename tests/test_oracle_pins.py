"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms, brute force
on tiny inputs, finite differences of independently written energies, invariants of the
implicit-Euler/quasi-Newton step (supplementary material, npFEM subsection), and the
paper's parameter table. None of these tests needs a GPU.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import npfem_inputs as I
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ct(kind=I.RBC, material=None, h=I.DT):
    x, t, mat = I.cell_type_inputs()[kind]
    return O.CellType(x, t, material or mat, h)


def _small(mesh_fn, material=None, h=I.DT, scale=1.0):
    x, t = mesh_fn()
    return O.CellType(scale * x, t, material or I.RBC_MATERIAL, h)


# ---------------------------------------------------------------- paper constants, meshes

def test_paper_parameter_table():
    p = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    m = I.RBC_MATERIAL
    assert (m.shear_B, m.area_C, m.skalak_D) == (p["skalak_B_pN_per_um"], p["skalak_C_pN_per_um"],
                                                 p["skalak_D_pN_per_um"])
    assert m.k_bend == p["k_bending_pN_um"] and m.k_vol == p["k_volume"]
    assert m.density == p["fluid_density_fg_per_um3"]
    xr, tr = I.rbc_mesh()
    xp, tp = I.platelet_mesh()
    assert xr.shape[0] == p["rbc_surface_vertices"] and xp.shape[0] == p["platelet_surface_vertices"]
    assert abs(I.PLT_DIAMETER - p["platelet_diameter_um"]) < 1e-12


def test_evans_fung_geometry():
    """Centre thickness R0*C0, ring radii R0 sin(theta), mesh volume near the analytic one."""
    from npfem_inputs.meshes import EF_R0, EF_C0, EF_C2, EF_C4
    x, t = I.rbc_mesh()
    assert abs((x[0, 2] - x[-1, 2]) - EF_R0 * EF_C0) < 1e-12
    r = np.hypot(x[1:-1, 0], x[1:-1, 1]).reshape(16, 16)
    th = np.pi * np.arange(1, 17) / 17
    assert np.allclose(r, EF_R0 * np.sin(th)[:, None], atol=1e-12)
    # analytic volume of the Evans-Fung body: 2 pi int_0^R0 r * 2 z(r) dr
    s = np.linspace(0, 1, 200001)
    rr = EF_R0 * np.sqrt(s)
    thick = EF_R0 * np.sqrt(1 - s) * (EF_C0 + EF_C2 * s + EF_C4 * s * s)
    vol = np.trapezoid(2 * np.pi * rr * thick * (EF_R0 / (2 * np.sqrt(np.maximum(s, 1e-300)))), s)
    summ = I.mesh_summary(x, t)
    assert 85.0 < summ["volume"] < vol and vol < 96.0          # inscribed polyhedron < body
    assert abs(summ["span_z"] - thick.max()) < 0.02
    assert abs(thick.max() - 2.566) < 2e-3
    assert (summ["n_triangles"], summ["n_edges"]) == (512, 768)
    xp, tp = I.platelet_mesh()
    sp = I.mesh_summary(xp, tp)
    assert (sp["n_triangles"], sp["n_edges"]) == (128, 192)
    assert abs(sp["span_z"] - 0.9) < 1e-12
    # ellipsoid volume 4/3 pi a^2 c bounds the inscribed mesh volume
    assert 0.8 * (4 / 3) * np.pi * 1.8 ** 2 * 0.45 < sp["volume"] < (4 / 3) * np.pi * 1.8 ** 2 * 0.45


# ---------------------------------------------------------------- rest frames and F

def test_deformation_gradient_reproduces_edges_and_stretch():
    ct = _ct()
    F0 = O.deformation_gradients(ct.X[None], ct)[0]
    # at rest F has orthonormal columns
    assert np.allclose(np.einsum("mdk,mdl->mkl", F0, F0), np.eye(2), atol=1e-12)
    rng = np.random.default_rng(3)
    x = ct.X + 0.05 * rng.normal(size=ct.X.shape)
    F = O.deformation_gradients(x[None], ct)[0]
    a, b, c = (ct.X[ct.tri[:, q]] for q in range(3))
    xa, xb, xc = (x[ct.tri[:, q]] for q in range(3))
    # F maps each rest edge (in the triangle's own plane) onto the deformed edge
    R0 = np.einsum("mdk,mdl->mkl", F0, np.stack([b - a, c - a], axis=-1))   # rest edges in 2D
    assert np.allclose(np.einsum("mdk,mkl->mdl", F, R0), np.stack([xb - xa, xc - xa], -1), atol=1e-12)
    # a flat triangle stretched by diag(s1, s2) after an in-plane rotation has sigma = (s1, s2)
    X = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.0], [0.4, 0.9, 0.0], [0, 0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 3, 1], [1, 3, 2], [0, 2, 3]])
    G, _ = O.triangle_rest_frames(X, tri)
    al = 0.7
    Rz = np.array([[np.cos(al), -np.sin(al), 0], [np.sin(al), np.cos(al), 0], [0, 0, 1]])
    xs = X @ (np.diag([1.3, 0.8, 1.0]) @ Rz).T
    Fs = np.einsum("jd,jk->dk", xs[tri[0]], G[0])
    assert np.allclose(np.sort(np.linalg.svd(Fs, compute_uv=False)), [0.8, 1.3], atol=1e-13)


# ---------------------------------------------------------------- projections

def _brute_area(s1, s2):
    h = lambda t: (t - s1) ** 2 + (1 / t - s2) ** 2
    ts = np.linspace(0.05, 5.0, 20001)
    t0 = ts[np.argmin(h(ts))]
    r = scipy.optimize.minimize_scalar(h, bracket=(t0 * 0.999, t0, t0 * 1.001), tol=1e-14)
    return r.x


def test_area_root_is_global_minimiser():
    rng = np.random.default_rng(0)
    s = np.sort(rng.uniform(0.3, 1.9, size=(200, 2)), axis=1)[:, ::-1]
    d = O.area_root(s[:, 0], s[:, 1])
    for (s1, s2), dd in zip(s, d):
        assert abs(dd - _brute_area(s1, s2)) < 1e-6
    # equal singular values below 2: the quartic factors as (t^2-1)(t^2-s t+1) -> t = 1
    eq = np.linspace(0.2, 1.95, 15)
    assert np.allclose(O.area_root(eq, eq), 1.0, atol=1e-12)


def test_strain_projection_closed_forms():
    ct = _ct()
    rng = np.random.default_rng(1)
    F = rng.normal(size=(1, 40, 3, 2))
    p_s, p_a = O.triangle_projections(F, ct)
    for f, p in zip(F[0], p_s[0]):
        ref = f @ np.linalg.inv(scipy.linalg.sqrtm(f.T @ f).real)   # polar factor F (F^T F)^-1/2
        assert np.allclose(p, ref, atol=1e-10)
    # area projection: det of the 2x2 stretch is one -> p_a has singular values (d, 1/d)
    sv = np.linalg.svd(p_a[0], compute_uv=False)
    assert np.allclose(sv[:, 0] * sv[:, 1], 1.0, atol=1e-12)
    # clamped strain limiting keeps F when the singular values are inside [s_min, s_max]
    mat = I.Material(strain_min=0.5, strain_max=2.0)
    ct2 = O.CellType(ct.X, ct.tri, mat, I.DT)
    Fin = np.stack([np.linalg.qr(rng.normal(size=(3, 2)))[0] @ np.diag([1.3, 0.7])
                    for _ in range(5)])[None]
    assert np.allclose(O.triangle_projections(Fin, ct2)[0], Fin, atol=1e-12)


def _hinge_geometric_u(x, H, i_k_area=True):
    """u = -sqrt(3/(A0+A1)) |e0| (n0 + n1), n the in-plane unit normals of the edge toward k, l."""
    i, j, k, l = (x[H[:, q]] for q in range(4))
    e0 = j - i
    def inward(p):
        w = p - i
        w = w - (np.einsum("ed,ed->e", w, e0) / np.einsum("ed,ed->e", e0, e0))[:, None] * e0
        return w / np.linalg.norm(w, axis=1)[:, None]
    A0 = 0.5 * np.linalg.norm(np.cross(e0, k - i), axis=1)
    A1 = 0.5 * np.linalg.norm(np.cross(e0, l - i), axis=1)
    return -(np.sqrt(3 / (A0 + A1)) * np.linalg.norm(e0, axis=1))[:, None] * (inward(k) + inward(l))


def test_bending_stencil_geometry():
    ct = _ct()
    assert np.allclose(ct.coef.sum(axis=1), 0.0, atol=1e-10)
    # the stencil applied to the rest shape equals the geometric edge-normal formula
    u = O.bending_vectors(ct.X[None], ct)[0]
    assert np.allclose(u, _hinge_geometric_u(ct.X, ct.hinge), atol=1e-11)
    # a coplanar hinge has u = 0
    X = np.array([[0, 0, 0], [1, 0.1, 0], [0.3, 0.8, 0], [0.5, -0.9, 0.0]], dtype=float)
    H = np.array([[0, 1, 2, 3]])
    i, j, k, l = X
    e0, e1, e2, e3, e4 = j - i, k - i, l - i, k - j, l - j
    cot = lambda a, b: a @ b / np.linalg.norm(np.cross(a, b))
    c01, c02, c03, c04 = cot(e0, e1), cot(e0, e2), cot(-e0, e3), cot(-e0, e4)
    coef = np.array([c03 + c04, c01 + c02, -c01 - c03, -c02 - c04])
    assert np.allclose(coef @ X, 0.0, atol=1e-14)


def test_volume_closed_forms_and_gradient():
    xt, tt = I.tetrahedron()
    assert abs(O.volume(xt[None], tt)[0] - 1 / 6) < 1e-15
    xo, to = I.octahedron(1.7)
    assert abs(O.volume(xo[None], to)[0] - 4 / 3 * 1.7 ** 3) < 1e-12
    xi, ti = I.icosahedron(1.0)
    a = np.linalg.norm(xi[0] - xi[11])
    assert abs(O.volume(xi[None], ti)[0] - 5 * (3 + 5 ** 0.5) / 12 * a ** 3) < 1e-12
    ct = _ct()
    rng = np.random.default_rng(2)
    x = ct.X + 0.1 * rng.normal(size=ct.X.shape)
    g = O.volume_gradient(x[None], ct.tri)[0]
    assert np.allclose(g.sum(axis=0), 0.0, atol=1e-12)
    eps = 1e-6
    for (i, d) in [(0, 2), (17, 0), (100, 1), (257, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd = (O.volume(xp[None], ct.tri)[0] - O.volume(xm[None], ct.tri)[0]) / (2 * eps)
        assert abs(fd - g[i, d]) < 1e-8


# ---------------------------------------------------------------- gradient and L

def _independent_energy(x, ct):
    """Elastic energy without the volume term, written from the definitions with no oracle
    projection code: singular values from eig(F^T F), area distance by brute minimisation,
    bending vectors as the rest stencil (pinned geometrically at rest) applied to x."""
    F = O.deformation_gradients(x[None], ct)[0]
    e = 0.0
    for t in range(ct.m):
        ev = np.linalg.eigvalsh(F[t].T @ F[t])
        s2, s1 = np.sqrt(np.maximum(ev, 0))
        c1, c2 = np.clip(s1, ct.s_min, ct.s_max), np.clip(s2, ct.s_min, ct.s_max)
        e += 0.5 * ct.w_s * ct.area[t] * ((s1 - c1) ** 2 + (s2 - c2) ** 2)
        h = lambda tt: (tt - s1) ** 2 + (1 / tt - s2) ** 2
        r = scipy.optimize.minimize_scalar(h, bracket=(0.5, 1.0, 2.0), tol=1e-14)
        e += 0.5 * ct.w_a * ct.area[t] * r.fun
    u = np.einsum("eq,eqd->ed", ct.coef, x[ct.hinge])
    e += 0.5 * ct.w_b * np.sum((np.linalg.norm(u, axis=1) - ct.rest_norm) ** 2)
    return e


def test_gradient_matches_finite_differences():
    mat = I.Material(shear_B=3.0, area_C=40.0, k_bend=2.0, k_vol=7.0)
    ct = _small(I.icosahedron, material=mat, scale=1.0)
    rng = np.random.default_rng(4)
    x = ct.X + 0.04 * rng.normal(size=ct.X.shape)
    y = ct.X + 0.03 * rng.normal(size=ct.X.shape)
    g = O.gradient(x[None], y[None], ct)[0]
    # inertia + independent elastic energy by central differences
    eps = 1e-6
    fd = np.zeros_like(x)
    for i in range(ct.n):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += eps
            xm[i, d] -= eps
            fd[i, d] = (_independent_energy(xp, ct) - _independent_energy(xm, ct)) / (2 * eps)
    fd += ct.mass / ct.h ** 2 * (x - y)
    # volume residual: -w_v lambda grad V with lambda (V0 - V)/|grad V|^2
    gV = O.volume_gradient(x[None], ct.tri)[0]
    lam = (ct.V0 - O.volume(x[None], ct.tri)[0]) / np.sum(gV * gV)
    fd += -ct.w_v * lam * gV
    assert np.allclose(g, fd, rtol=0, atol=2e-6 * np.abs(g).max())


def test_system_matrix_is_hessian_of_quadratic_part():
    """d^T L d = 2 Q(d) with Q written from the energies: inertia, volume weight, ||F||^2
    terms (F from a rest frame built on the other edge) and the bending vectors."""
    ct = _ct()
    assert np.allclose(ct.L, ct.L.T)
    assert np.all(np.linalg.eigvalsh(ct.L) > 0)
    X, tri = ct.X, ct.tri
    a, b, c = X[tri[:, 0]], X[tri[:, 1]], X[tri[:, 2]]
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.normal(size=X.shape)
        q = 0.5 * (ct.mass / ct.h ** 2 + ct.w_v) * np.sum(d * d)
        for t in range(ct.m):
            # frame on edge ac: rest edges in 2D, F = D_s D_m^-1 with D_s = [d_b - d_a, d_c - d_a]
            e1, e2 = c[t] - a[t], b[t] - a[t]
            t1 = e1 / np.linalg.norm(e1)
            t2 = e2 - (e2 @ t1) * t1
            t2 /= np.linalg.norm(t2)
            Dm = np.array([[e2 @ t1, e1 @ t1], [e2 @ t2, e1 @ t2]])
            Ds = np.stack([d[tri[t, 1]] - d[tri[t, 0]], d[tri[t, 2]] - d[tri[t, 0]]], 1)
            F = Ds @ np.linalg.inv(Dm)
            q += 0.5 * (ct.w_s + ct.w_a) * ct.area[t] * np.sum(F * F)
        u = np.einsum("eq,eqd->ed", ct.coef, d[ct.hinge])
        q += 0.5 * ct.w_b * np.sum(u * u)
        dv = d.reshape(ct.n, 3)
        assert abs(np.einsum("id,ij,jd->", dv, ct.L, dv) - 2 * q) < 1e-9 * abs(2 * q)


# ---------------------------------------------------------------- step invariants

def _place(ct, rng):
    R = I.random_rotations(rng, 1)[0]
    return ct.X @ R.T + rng.uniform(0, 50, size=3), R


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
def test_rest_shape_is_fixed_point(kind):
    ct = _ct(kind)
    rng = np.random.default_rng(6)
    x, _ = _place(ct, rng)
    z = np.zeros_like(x)[None]
    for K in (0, 1, 10):
        xn, vn = O.step(ct, x[None], z, z, K)
        assert np.abs(xn[0] - x).max() < 1e-12
        assert np.abs(vn).max() < 1e-10


def test_ballistic_closed_form():
    ct = _ct()
    rng = np.random.default_rng(7)
    x = ct.X[None] + 0.02 * rng.normal(size=(1,) + ct.X.shape)
    v = rng.normal(size=x.shape)
    f = rng.normal(size=x.shape)
    y = x + ct.h * v + ct.h ** 2 * f / ct.mass
    xn, vn = O.step(ct, x, v, f, 0)
    assert np.array_equal(xn, y)
    free = O.CellType(ct.X, ct.tri, I.Material(shear_B=0, area_C=0, k_bend=0, k_vol=0), ct.h)
    xn, vn = O.step(free, x, v, f, 10)
    assert np.allclose(xn, y, atol=1e-13)
    assert np.allclose(vn, (y - x) / ct.h, atol=1e-11)


def test_rigid_uniform_acceleration():
    ct = _ct()
    acc = np.array([0.3, -1.1, 0.7])
    v0 = np.array([1.0, 2.0, -0.5])
    x = ct.X[None]
    v = np.broadcast_to(v0, x.shape).copy()
    f = np.broadcast_to(ct.mass * acc, x.shape).copy()
    xn, vn = O.step(ct, x, v, f, 10)
    assert np.allclose(xn[0], ct.X + ct.h * v0 + ct.h ** 2 * acc, atol=1e-12)


@pytest.mark.parametrize("K", [1, 3, 10])
def test_linear_momentum(K):
    ct = _ct()
    rng = np.random.default_rng(8)
    x = ct.X[None] + 0.05 * rng.normal(size=(1,) + ct.X.shape)
    v = rng.normal(size=x.shape)
    f = 50 * rng.normal(size=x.shape)
    xn, vn = O.step(ct, x, v, f, K)
    lhs = ct.mass * (xn - x).sum(axis=1)
    rhs = ct.h * ct.mass * v.sum(axis=1) + ct.h ** 2 * f.sum(axis=1)
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())


def test_rigid_motion_invariance():
    ct = _ct(I.PLT)
    rng = np.random.default_rng(9)
    x = ct.X[None] + 0.02 * rng.normal(size=(1,) + ct.X.shape)
    v = rng.normal(size=x.shape)
    f = 20 * rng.normal(size=x.shape)
    R = I.random_rotations(rng, 1)[0]
    tr = np.array([10.0, -4.0, 3.0])
    xn, vn = O.step(ct, x, v, f, 10)
    xr, vr = O.step(ct, x @ R.T + tr, v @ R.T, f @ R.T, 10)
    assert np.abs(xr - (xn @ R.T + tr)).max() < 1e-11
    assert np.abs(vr - vn @ R.T).max() < 1e-9


@pytest.mark.parametrize("k_vol", [0.0, 250.0])
def test_energy_non_increasing(k_vol):
    """Local/global alternation cannot increase g (exact projections); with the linearised
    volume projection the slack is second order, checked at 1e-12 relative."""
    ct = O.CellType(*I.rbc_mesh(), I.Material(k_vol=k_vol), I.DT)
    rng = np.random.default_rng(10)
    x = ct.X[None]
    v = np.zeros_like(x)
    f = 1000.0 * rng.normal(size=x.shape)
    hist = []
    O.step(ct, x, v, f, 10, history=hist)
    y = O.predict(x, v, f, ct)
    e = [O.energy(h, y, ct)[0] for h in hist]
    for a, b in zip(e, e[1:]):
        assert b <= a * (1 + 1e-12)
    assert e[-1] < e[0]


@pytest.mark.parametrize("mesh", ["tet", "oct", "ico", "rbc", "plt"])
def test_prefactored_solve_equals_dense_solve(mesh):
    if mesh in ("rbc", "plt"):
        ct = _ct(I.RBC if mesh == "rbc" else I.PLT)
    else:
        fn = {"tet": I.tetrahedron, "oct": I.octahedron, "ico": I.icosahedron}[mesh]
        ct = _small(fn)
    rng = np.random.default_rng(11)
    b = rng.normal(size=(4, ct.n, 3))
    xc = O.solve(ct, b, "cholesky")
    xd = O.solve(ct, b, "dense")
    # brute force: Gauss-Jordan on the augmented system, no library solve
    A = np.concatenate([ct.L, np.transpose(b, (1, 0, 2)).reshape(ct.n, -1)], axis=1)
    for col in range(ct.n):
        p = col + np.argmax(np.abs(A[col:, col]))
        A[[col, p]] = A[[p, col]]
        A[col] /= A[col, col]
        for r in range(ct.n):
            if r != col:
                A[r] -= A[r, col] * A[col]
    xg = np.transpose(A[:, ct.n:].reshape(ct.n, 4, 3), (1, 0, 2))
    scale = np.abs(xg).max()
    assert np.abs(xc - xd).max() <= 1e-13 * scale
    assert np.abs(xc - xg).max() <= 1e-12 * scale


def test_quasi_newton_equals_projective_dynamics():
    ct = _ct()
    rng = np.random.default_rng(12)
    x = ct.X[None] + 0.02 * rng.normal(size=(1,) + ct.X.shape)
    v = rng.normal(size=x.shape)
    f = 100 * rng.normal(size=x.shape)
    xq, _ = O.step(ct, x, v, f, 10, form="qn")
    xp, _ = O.step(ct, x, v, f, 10, form="pd")
    assert np.abs(xq - xp).max() < 1e-12


def test_iteration_converges_to_newtons_law():
    ct = _ct()
    rng = np.random.default_rng(13)
    x = ct.X[None]
    v = np.zeros_like(x)
    f = 200 * rng.normal(size=x.shape)
    y = O.predict(x, v, f, ct)
    g0 = np.abs(O.gradient(y, y, ct)).max()
    xk, _ = O.step(ct, x, v, f, 60)
    assert np.abs(O.gradient(xk, y, ct)).max() < 1e-9 * g0


def test_single_step_discriminates_iteration_count():
    """A 200 pN kick separates K = 9 from K = 10 by well above 1e-7 of the diameter."""
    ct = _ct()
    rng = np.random.default_rng(14)
    x = ct.X[None]
    v = np.zeros_like(x)
    f = 200 * rng.normal(size=x.shape)
    x9, _ = O.step(ct, x, v, f, 9)
    x10, _ = O.step(ct, x, v, f, 10)
    assert np.abs(x9 - x10).max() / I.RBC_DIAMETER > 2e-7


@pytest.mark.parametrize("kind", [I.RBC, I.PLT])
def test_lumped_mass_is_total_mass(kind):
    """The lumped mass matrix carries the body's total mass (membrane + interior fluid):
    n m = density * enclosed volume, with the volume from the plain mesh summary."""
    x, t, mat = I.cell_type_inputs()[kind]
    ct = O.CellType(x, t, mat, I.DT)
    vol = I.mesh_summary(x, t)["volume"]
    assert abs(ct.n * ct.mass - mat.density * vol) < 1e-9 * mat.density * vol
    # the system matrix diagonal carries m/h^2 + k_vol on top of non-negative stiffness terms
    assert np.all(np.diag(ct.L) >= ct.mass / ct.h ** 2 + ct.w_v - 1e-9)


# ------------------------------------------------------------ position-based damping (PBD)


def _cloud(seed, kind=I.RBC, n_cells=3):
    ct = _ct(kind)
    rng = np.random.default_rng(seed)
    x = ct.X[None] + 0.1 * rng.normal(size=(n_cells,) + ct.X.shape) + rng.normal(size=(n_cells, 1, 3)) * 20
    return ct, x, rng


def test_pbd_damping_keeps_rigid_velocity_fields():
    """v = a + w0 x (x - c) (any a, w0, c) is already rigid: damping leaves it unchanged."""
    ct, x, rng = _cloud(31)
    a = rng.normal(size=(3, 1, 3))
    w0 = rng.normal(size=(3, 1, 3))
    c = rng.normal(size=(3, 1, 3)) * 5
    v = a + np.cross(w0, x - c)
    for kappa in (0.3, 0.8, 1.0):
        assert np.allclose(O.pbd_damp(x, v, kappa), v, atol=1e-11 * np.abs(v).max())


def test_pbd_damping_conserves_linear_and_angular_momentum():
    """sum v and sum (x - x_cm) x v (equal masses) are unchanged for any kappa."""
    ct, x, rng = _cloud(32)
    v = rng.normal(size=x.shape)
    xcm = x.mean(axis=1, keepdims=True)
    for kappa in (0.5, 0.9):
        vd = O.pbd_damp(x, v, kappa)
        assert np.allclose(vd.sum(axis=1), v.sum(axis=1), atol=1e-10)
        assert np.allclose(np.cross(x - xcm, vd).sum(axis=1), np.cross(x - xcm, v).sum(axis=1),
                           atol=1e-9)
        # and the non-rigid part shrinks by exactly 1 - kappa
        rig = O.pbd_damp(x, v, 1.0)
        assert np.allclose(vd - rig, (1 - kappa) * (v - rig), atol=1e-10)


def test_pbd_angular_velocity_is_the_least_squares_rigid_fit():
    """w = I^-1 L is the angular velocity of the least-squares rigid fit of v, found here
    independently with a generic least-squares solve of v - v_cm = w x r = -[r]_x w."""
    ct, x, rng = _cloud(33, kind=I.PLT, n_cells=2)
    v = rng.normal(size=x.shape)
    vcm, w, xcm = O.rigid_velocity_fit(x, v)
    for c in range(x.shape[0]):
        r = x[c] - x[c].mean(axis=0)
        A = np.zeros((3 * ct.n, 3))
        for i in range(ct.n):
            rx, ry, rz = r[i]
            A[3 * i:3 * i + 3] = -np.array([[0, -rz, ry], [rz, 0, -rx], [-ry, rx, 0]])
        b = (v[c] - v[c].mean(axis=0)).ravel()
        w_ls = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.allclose(w[c], w_ls, rtol=1e-10, atol=1e-12)
        assert np.allclose(vcm[c], v[c].mean(axis=0))


def test_pbd_damping_with_kappa_one_is_idempotent():
    ct, x, rng = _cloud(34)
    v = rng.normal(size=x.shape)
    v1 = O.pbd_damp(x, v, 1.0)
    assert np.allclose(O.pbd_damp(x, v1, 1.0), v1, atol=1e-11)
    assert np.allclose(O.pbd_damp(x, v1, 0.6), v1, atol=1e-11)


def test_damped_step_conserves_linear_momentum_and_reduces_to_undamped():
    """With kappa = 0 the step is the undamped one; with kappa > 0 the prediction's
    velocity keeps sum m v, so sum m (x_{n+1} - x_n) = h sum m v_n + h^2 sum F still holds."""
    x0, t0, mat = I.cell_type_inputs()[I.RBC]
    ct0 = O.CellType(x0, t0, mat, I.DT)
    ctk = O.CellType(x0, t0, mat.with_kappa(0.8), I.DT)
    ctz = O.CellType(x0, t0, mat.with_kappa(0.0), I.DT)
    rng = np.random.default_rng(35)
    x = ct0.X[None] + 0.05 * rng.normal(size=(1,) + ct0.X.shape)
    v = rng.normal(size=x.shape)
    f = 50 * rng.normal(size=x.shape)
    xa, _ = O.step(ct0, x, v, f, 5)
    xz, _ = O.step(ctz, x, v, f, 5)
    assert np.array_equal(xa, xz)
    xk, vk = O.step(ctk, x, v, f, 5)
    lhs = ctk.mass * (xk - x).sum(axis=1)
    rhs = ctk.h * ctk.mass * v.sum(axis=1) + ctk.h ** 2 * f.sum(axis=1)
    assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())
    assert np.abs(xk - xa).max() > 1e-4        # damping changes the result


# ------------------------------------------------- boundary filters: median of F, velocity cap


def test_median_filter_constant_field_and_isolated_spike():
    """A constant force field passes unchanged; a spike on one vertex (all others zero) is
    removed everywhere, since no closed one ring holds it more than once."""
    ct = _ct(I.RBC)
    f = np.broadcast_to(np.array([1.5, -2.0, 0.25]), (1, ct.n, 3)).copy()
    assert np.array_equal(O.median_filter_forces(f, ct), f)
    g = np.zeros((1, ct.n, 3))
    g[0, 37] = [1e3, -5e2, 7e2]
    assert np.array_equal(O.median_filter_forces(g, ct), np.zeros_like(g))


def test_median_filter_brute_force_small_meshes():
    """On the octahedron each vertex's closed ring has 5 members (odd count), on the
    tetrahedron 4 (even: mean of the two middle values); compared with a sort done here."""
    rng = np.random.default_rng(41)
    for mesh_fn in (I.octahedron, I.tetrahedron):
        x, t = mesh_fn()
        ct = O.CellType(x, t, I.RBC_MATERIAL, I.DT)
        f = rng.normal(size=(2, ct.n, 3))
        out = O.median_filter_forces(f, ct)
        for i in range(ct.n):
            members = {i} | {int(u) for tr in t for u in tr if i in tr}
            vals = np.sort(f[:, sorted(members), :], axis=1)
            k = len(members)
            ref = vals[:, k // 2, :] if k % 2 else 0.5 * (vals[:, k // 2 - 1, :] + vals[:, k // 2, :])
            assert np.allclose(out[:, i, :], ref), (mesh_fn.__name__, i)


def test_velocity_cap():
    rng = np.random.default_rng(42)
    v = rng.normal(size=(2, 50, 3)) * 3
    c = O.cap_velocities(v, 2.0)
    s, sc = np.linalg.norm(v, axis=-1), np.linalg.norm(c, axis=-1)
    assert np.all(sc <= 2.0 + 1e-12)
    assert np.array_equal(c[s <= 2.0], v[s <= 2.0])
    fast = s > 2.0
    # direction kept
    assert np.allclose(c[fast] / sc[fast][:, None], v[fast] / s[fast][:, None])
    assert np.array_equal(O.cap_velocities(v, 0.0), v)


def test_step_caps_velocities_and_keeps_positions():
    """A type with v_max returns the uncapped step's positions and the uncapped velocities
    scaled to length v_max where they were longer (a kicked cell moves faster than the cap)."""
    x0, t, m = I.cell_type_inputs()[I.PLT]
    ct = O.CellType(x0, t, m, I.DT)
    ctc = O.CellType(x0, t, m.with_v_max(0.05), I.DT)
    rng = np.random.default_rng(47)
    x = x0[None] + 0.02 * rng.normal(size=(1,) + x0.shape)
    v = 0.05 * rng.normal(size=x.shape)
    f = 0.0 * x
    xa, va = O.step(ct, x, v, f, 3)
    xb, vb = O.step(ctc, x, v, f, 3)
    assert np.array_equal(xa, xb)
    s = np.linalg.norm(va, axis=-1)
    assert np.any(s > 0.05) and np.any(s <= 0.05)
    assert np.array_equal(vb[s <= 0.05], va[s <= 0.05])
    fast = s > 0.05
    assert np.allclose(np.linalg.norm(vb[fast], axis=-1), 0.05, rtol=1e-14)
    assert np.allclose(vb[fast] * (s[fast] / 0.05)[:, None], va[fast], rtol=1e-12)


# ------------------------------------------------------------------ Rayleigh damping (f1)


def _deformed_plt(seed, amp=0.03):
    x0, t, m = I.cell_type_inputs()[I.PLT]
    rng = np.random.default_rng(seed)
    return x0, t, m, x0[None] + amp * rng.normal(size=(1,) + x0.shape)


def test_rayleigh_free_flight_closed_form():
    """With alpha only, M~ = (1 + h alpha) M, so the prediction (K = 0 iterations) is
    y = x + (h v + h^2 F/m) / (1 + h alpha), straight from the definitions of M~ and y_n."""
    x0, t, m, x = _deformed_plt(60)
    alpha = 0.7
    ct = O.CellType(x0, t, m.with_rayleigh(alpha, 0.0), I.DT)
    rng = np.random.default_rng(61)
    v, f = rng.normal(size=x.shape), 30.0 * rng.normal(size=x.shape)
    y, _ = O.step(ct, x, v, f, 0)
    ref = x + (I.DT * v + I.DT ** 2 * f / ct.mass) / (1.0 + I.DT * alpha)
    assert np.allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_rayleigh_keeps_rigid_translation():
    """K annihilates a uniform translation (sum_j g_j = 0, sum_q a_q = 0), so beta damping
    leaves a cell translating at rest shape exactly on its free-flight path."""
    x0, t, m = I.cell_type_inputs()[I.RBC]
    ct = O.CellType(x0, t, m.with_rayleigh(0.0, 0.05), I.DT)
    u = np.array([0.3, -0.2, 0.5])
    x = x0[None] + 10.0
    v = np.broadcast_to(u, x.shape).copy()
    x1, v1 = O.step(ct, x, v, 0 * x, 5)
    assert np.abs(x1 - (x + I.DT * u)).max() <= 1e-11
    assert np.abs(v1 - u).max() <= 1e-9
    assert np.abs(ct.K.sum(axis=1)).max() <= 1e-9 * np.abs(ct.K).max()


def test_rayleigh_converged_step_satisfies_newtons_law():
    """A converged damped step solves the implicit-Euler equation of motion with
    C = alpha M + beta K: F_int(x1) + F_ext - C v1 = M (v1 - v0)/h. F_int comes from an
    undamped type (gradient at y = x has no mass term) and K from its system matrix minus the
    mass and volume diagonal, so neither shares the damped type's M~ or y_n."""
    x0, t, m, x = _deformed_plt(62, amp=0.02)
    alpha, beta = 0.3, 0.05
    ct = O.CellType(x0, t, m.with_rayleigh(alpha, beta), I.DT)
    ct0 = O.CellType(x0, t, m, I.DT)
    rng = np.random.default_rng(63)
    v0, f = 0.05 * rng.normal(size=x.shape), 20.0 * rng.normal(size=x.shape)
    x1, v1 = O.step(ct, x, v0, f, 200)
    K = ct0.L - np.eye(ct0.n) * (ct0.mass / ct0.h ** 2 + ct0.w_v)
    f_int = -O.gradient(x1, x1, ct0)
    Cv = alpha * ct0.mass * v1 + beta * np.einsum("ij,njd->nid", K, v1)
    res = f_int + f - Cv - ct0.mass * (v1 - v0) / I.DT
    scale = np.abs(ct0.mass * (v1 - v0) / I.DT).max() + np.abs(f).max()
    assert np.abs(res).max() <= 1e-10 * scale, np.abs(res).max() / scale   # 5e-13 here
    # and damping matters at this size: the undamped step differs by more than the step
    xu, _ = O.step(ct0, x, v0, f, 200)
    assert np.abs(xu - x1).max() > 0.5 * np.abs(x1 - x).max()


def test_rayleigh_quasi_newton_equals_projective_dynamics():
    """x - L~^-1 grad g(x) = L~^-1 rhs(x) with the damped M~ in both g and rhs."""
    x0, t, m, x = _deformed_plt(64)
    ct = O.CellType(x0, t, m.with_rayleigh(0.2, 0.03), I.DT)
    rng = np.random.default_rng(65)
    v, f = 0.05 * rng.normal(size=x.shape), 10.0 * rng.normal(size=x.shape)
    a, _ = O.step(ct, x, v, f, 4, form="qn")
    b, _ = O.step(ct, x, v, f, 4, form="pd")
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


# ------------------------------------------------------- collision energies (PIK, f2 part)


def _contacts(x, seed, frac=0.15, w=400.0, gap=0.3):
    rng = np.random.default_rng(seed)
    N, n, _ = x.shape
    wc = np.where(rng.random((N, n)) < frac, w, 0.0)
    pc = x + gap * rng.normal(size=x.shape)
    return pc, wc


def test_contacts_with_zero_weight_change_nothing():
    x0, t, m, x = _deformed_plt(80)
    ct = O.CellType(x0, t, m, I.DT)
    rng = np.random.default_rng(81)
    v, f = 0.05 * rng.normal(size=x.shape), 10.0 * rng.normal(size=x.shape)
    pc, _ = _contacts(x, 82)
    a, va = O.step(ct, x, v, f, 6)
    b, vb = O.step(ct, x, v, f, 6, contacts=(pc, np.zeros(x.shape[:2])))
    assert np.array_equal(a, b) and np.array_equal(va, vb)


def test_converged_step_with_contacts_satisfies_newtons_law():
    """At convergence the contact energies act as forces -w (x1 - p) in the implicit-Euler
    equation of motion: F_int(x1) + F_ext - w (x1 - p) = M (v1 - v0)/h, with F_int from the
    gradient at y = x (no mass term, no contacts) and the contact force written out here."""
    x0, t, m = I.cell_type_inputs()[I.RBC]
    x = x0[None] + 0.02 * np.random.default_rng(83).normal(size=(1,) + x0.shape)
    ct = O.CellType(x0, t, m, I.DT)
    rng = np.random.default_rng(84)
    v0, f = 0.05 * rng.normal(size=x.shape), 10.0 * rng.normal(size=x.shape)
    pc, wc = _contacts(x, 85, gap=0.1)
    x1, v1 = O.step(ct, x, v0, f, 100, contacts=(pc, wc))
    res = -O.gradient(x1, x1, ct) + f - wc[..., None] * (x1 - pc) - ct.mass * (v1 - v0) / I.DT
    scale = np.abs(ct.mass * (v1 - v0) / I.DT).max() + np.abs(f).max()
    assert np.abs(res).max() <= 1e-10 * scale, np.abs(res).max() / scale   # 5e-14 here
    # the contacts pull: every contacting vertex ends closer to its point than without them
    xf, _ = O.step(ct, x, v0, f, 100)
    on = wc > 0
    assert np.all(np.linalg.norm(x1 - pc, axis=-1)[on] < np.linalg.norm(xf - pc, axis=-1)[on])


# --------------------------------------------------- Skalak membrane with line search (f2)


def _skalak_ct(kind=I.RBC):
    x0, t, m = I.cell_type_inputs()[kind]
    return x0, t, O.CellType(x0, t, m.with_membrane("skalak"), I.DT)


def test_skalak_density_closed_forms():
    """Equibiaxial stretch l (C = l^2 1): W = (B/2)(l^2 - 1)^2 + (C/4)(l^4 - 1)^2; uniaxial
    (l, 1): W = ((B + C)/4)(l^2 - 1)^2; at rest W = 0 and dW/dF = 0 (worked by hand from the
    invariants)."""
    _, _, ct = _skalak_ct()
    B, C = ct.w_s, ct.w_a
    for lam in (0.8, 1.0, 1.03, 1.5):
        Fe = np.zeros((1, 1, 3, 2)); Fe[0, 0, 0, 0] = Fe[0, 0, 1, 1] = lam
        W, P = O.skalak_density(Fe, ct)
        assert np.isclose(W[0, 0], 0.5 * B * (lam ** 2 - 1) ** 2 + 0.25 * C * (lam ** 4 - 1) ** 2, rtol=1e-13, atol=1e-300)
        Fu = np.zeros((1, 1, 3, 2)); Fu[0, 0, 0, 0] = lam; Fu[0, 0, 1, 1] = 1.0
        Wu, _ = O.skalak_density(Fu, ct)
        assert np.isclose(Wu[0, 0], 0.25 * (B + C) * (lam ** 2 - 1) ** 2, rtol=1e-13, atol=1e-300)
        if lam == 1.0:
            assert W[0, 0] == 0.0 and np.abs(P).max() == 0.0


def test_skalak_stress_matches_finite_differences():
    _, _, ct = _skalak_ct()
    rng = np.random.default_rng(90)
    F = np.zeros((1, 5, 3, 2))
    F[0, :, 0, 0] = F[0, :, 1, 1] = 1.0
    F += 0.2 * rng.normal(size=F.shape)
    _, P = O.skalak_density(F, ct)
    h = 1e-6
    for d in range(3):
        for k in range(2):
            Fp, Fm = F.copy(), F.copy()
            Fp[..., d, k] += h
            Fm[..., d, k] -= h
            fd = (O.skalak_density(Fp, ct)[0] - O.skalak_density(Fm, ct)[0]) / (2 * h)
            assert np.allclose(P[..., d, k], fd, rtol=1e-6, atol=1e-6 * np.abs(P).max())


def test_skalak_line_search_decreases_g_every_iteration():
    """The Armijo rule makes every iteration a descent step of g (with its projections)."""
    x0, t, ct = _skalak_ct()
    rng = np.random.default_rng(91)
    x = x0[None] + 0.03 * rng.normal(size=(2,) + x0.shape)
    v, f = 0.1 * rng.normal(size=x.shape), 200.0 * rng.normal(size=x.shape)
    y = O.predict(x, v, f, ct)
    xk, g_prev = y.copy(), O.energy(y, y, ct)
    for _ in range(10):
        xk = O.line_search_update(ct, xk, y)
        g_now = O.energy(xk, y, ct)
        assert np.all(g_now <= g_prev + 1e-12 * np.abs(g_prev))
        g_prev = g_now
    # an inflated cell (area strain ~ 1): the full step overshoots and is halved, still descent
    xi = (1.4 * x0)[None]
    y = xi.copy()
    xk, g_prev, halved = y.copy(), O.energy(y, y, ct), False
    for _ in range(4):
        gk = O.gradient(xk, y, ct)
        d = -O.solve(ct, gk)
        full = O.energy(xk + d, y, ct) > g_prev + O.ARMIJO_C * np.einsum("nid,nid->n", gk, d)
        halved |= bool(full.any())
        xk = O.line_search_update(ct, xk, y)
        g_now = O.energy(xk, y, ct)
        assert np.all(g_now < g_prev)
        g_prev = g_now
    assert halved


def test_skalak_rigid_invariance_and_newtons_law():
    """A rotated and translated problem gives the rotated and translated step; a converged
    step satisfies the equation of motion with F_int = -grad of the Skalak, bending and volume
    energies."""
    x0, t, ct = _skalak_ct()
    rng = np.random.default_rng(92)
    x = x0[None] + 0.02 * rng.normal(size=(1,) + x0.shape)
    v, f = 0.05 * rng.normal(size=x.shape), 10.0 * rng.normal(size=x.shape)
    R = I.random_rotations(np.random.default_rng(93), 1)[0]
    tr = np.array([3.0, -2.0, 5.0])
    a, _ = O.step(ct, x, v, f, 8)
    b, _ = O.step(ct, x @ R.T + tr, v @ R.T, f @ R.T, 8)
    assert np.abs(b - (a @ R.T + tr)).max() <= 1e-11
    x1, v1 = O.step(ct, x, v, f, 150)
    res = -O.gradient(x1, x1, ct) + f - ct.mass * (v1 - v) / I.DT
    scale = np.abs(ct.mass * (v1 - v) / I.DT).max() + np.abs(f).max()
    assert np.abs(res).max() <= 1e-9 * scale, np.abs(res).max() / scale


# ---------------------------------------------------------------- objective g, area, line search

def _fd_energy_gradient(x, y, ct, contacts, eps):
    fd = np.zeros_like(x)
    for i in range(x.shape[1]):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[0, i, d] += eps
            xm[0, i, d] -= eps
            fd[0, i, d] = (O.energy(xp, y, ct, contacts)[0] - O.energy(xm, y, ct, contacts)[0]) / (2 * eps)
    return fd


@pytest.mark.parametrize("membrane", ["pd", "skalak"])
@pytest.mark.parametrize("rayleigh", [False, True])
def test_energy_is_the_potential_of_the_pinned_gradient(membrane, rayleigh):
    """g(x) of the minimisation form (npFEM subsection) against the gradient, which is pinned by
    finite differences of an independently written energy: with the volume weight at zero every
    remaining term of g (inertia with M or the Rayleigh M~, strain + area or the Skalak
    membrane, bending, collision energies) is exactly the potential of its gradient term, so
    the central difference of energy() must reproduce gradient() (a wrong factor on any term of
    either side fails)."""
    mat = I.Material(shear_B=3.0, area_C=40.0, k_bend=2.0, k_vol=0.0, membrane=membrane)
    if rayleigh:
        mat = mat.with_rayleigh(0.3, 0.05)
    ct = _small(I.icosahedron, material=mat)
    rng = np.random.default_rng(301)
    x = (ct.X + 0.05 * rng.normal(size=ct.X.shape))[None]
    y = (ct.X + 0.04 * rng.normal(size=ct.X.shape))[None]
    w = np.where(rng.random(ct.n) < 0.4, 60.0, 0.0)[None]
    p = x + 0.1 * rng.normal(size=x.shape)
    g = O.gradient(x, y, ct, (p, w))
    fd = _fd_energy_gradient(x, y, ct, (p, w), 1e-6)
    rel = np.abs(fd - g).max() / np.abs(g).max()
    assert rel <= 1e-6, rel
    # the collision term alone: w (x - p) is the gradient of (w/2)|x - p|^2
    e_c = O.energy(x, y, ct, (p, w))[0] - O.energy(x, y, ct)[0]
    assert np.isclose(e_c, 0.5 * np.sum(w[0] * np.sum((x[0] - p[0]) ** 2, axis=1)), rtol=1e-12)


def test_energy_volume_term_is_the_linearised_projection_distance():
    """The volume term of g is (k_vol/2)|x - p_vol|^2 with p_vol = x + lambda grad V, i.e.
    (k_vol/2)(V0 - V)^2/|grad V|^2, with V and grad V from the closed-form-pinned volume and
    volume_gradient (the term is not the potential of its gradient term, so it is pinned on its
    own)."""
    base = dict(shear_B=3.0, area_C=40.0, k_bend=2.0)
    ct0 = _small(I.icosahedron, material=I.Material(k_vol=0.0, **base))
    ct1 = _small(I.icosahedron, material=I.Material(k_vol=7.0, **base))
    rng = np.random.default_rng(302)
    x = (ct0.X * 1.05 + 0.05 * rng.normal(size=ct0.X.shape))[None]
    y = ct0.X[None]
    dV = ct1.V0 - O.volume(x, ct1.tri)[0]
    gV = O.volume_gradient(x, ct1.tri)[0]
    expect = 0.5 * 7.0 * dV ** 2 / np.sum(gV * gV)
    got = O.energy(x, y, ct1)[0] - O.energy(x, y, ct0)[0]
    assert abs(dV) > 1e-3 * ct1.V0
    assert np.isclose(got, expect, rtol=1e-12), (got, expect)


def test_surface_area_closed_forms():
    """Total area of the platonic meshes from their edge length a: tetrahedron corner (three
    right isosceles faces of legs 1 plus an equilateral face of side sqrt 2), regular
    octahedron 2 sqrt(3) a^2, regular icosahedron 5 sqrt(3) a^2; a scaled mesh scales as s^2;
    a rigid motion keeps it."""
    xt, tt = I.tetrahedron()
    assert np.isclose(O.surface_area(xt[None], tt)[0], 1.5 + 3 ** 0.5 / 2, rtol=1e-14)
    xo, to = I.octahedron(1.7)
    a = np.linalg.norm(xo[0] - xo[1])
    assert np.isclose(O.surface_area(xo[None], to)[0], 2 * 3 ** 0.5 * a * a, rtol=1e-14)
    xi, ti = I.icosahedron(1.3)
    a = min(np.linalg.norm(xi[0] - xi[j]) for j in range(1, 12))
    assert np.isclose(O.surface_area(xi[None], ti)[0], 5 * 3 ** 0.5 * a * a, rtol=1e-13)
    R = I.random_rotations(np.random.default_rng(303), 1)[0]
    moved = (2.5 * xi) @ R.T + np.array([10.0, -4.0, 7.0])
    assert np.isclose(O.surface_area(moved[None], ti)[0], 2.5 ** 2 * 5 * 3 ** 0.5 * a * a, rtol=1e-13)


def test_line_search_step_lengths_closed_form():
    """One line-searched iteration where g along the direction is a known quadratic: elastic
    weights zero and every vertex in contact with weight w, started at x = y. Then L = (m/h^2) I,
    the direction is d = -c (y - p) with c = w h^2/m, and
    g(y + a d) = (w S/2)(1 - 2 a c + a^2 c (1 + c)), S = sum |y - p|^2, with slope -c w S, so
    the Armijo test (constant 1e-4) holds exactly for a <= 2 (1 - 1e-4)/(1 + c). Cells with
    c = 0.5, 1.5, 3, 5 and 1000 must take 1, 1/2, 1/4 (1/2 misses the bound 0.49995 by the
    Armijo constant alone), 1/4 and the smallest step 1/256 (none qualifies)."""
    mat = I.Material(shear_B=0.0, area_C=0.0, k_bend=0.0, k_vol=0.0, membrane="skalak")
    ct = _small(I.icosahedron, material=mat)
    cs = np.array([0.5, 1.5, 3.0, 5.0, 1000.0])
    expect = np.array([1.0, 0.5, 0.25, 0.25, 1.0 / 256])
    rng = np.random.default_rng(304)
    N = len(cs)
    y = np.broadcast_to(ct.X, (N, ct.n, 3)) + 0.01 * rng.normal(size=(N, ct.n, 3))
    p = y + 0.2 * rng.normal(size=y.shape)
    w = np.broadcast_to((cs * ct.mass / ct.h ** 2)[:, None], (N, ct.n)).copy()
    x1 = O.line_search_update(ct, y.copy(), y, (p, w))
    a = (x1 - y) / (-cs[:, None, None] * (y - p))
    assert np.allclose(a, expect[:, None, None], rtol=1e-9, atol=0), a[:, 0, 0]


# ---------------------------------------------------------------- planted mistakes
# Each case plants a mistake in the oracle (a helper or constant of its module, patched for the
# test only) and checks that the pin above that covers it fails.

import oracle.npfem_oracle as OM   # noqa: E402  (the module whose globals the oracle reads)

def _energy_gradient_mismatch(membrane="skalak"):
    mat = I.Material(shear_B=3.0, area_C=40.0, k_bend=2.0, k_vol=0.0, membrane=membrane)
    ct = _small(I.icosahedron, material=mat)
    rng = np.random.default_rng(301)
    x = (ct.X + 0.05 * rng.normal(size=ct.X.shape))[None]
    y = (ct.X + 0.04 * rng.normal(size=ct.X.shape))[None]
    g = O.gradient(x, y, ct)
    fd = _fd_energy_gradient(x, y, ct, None, 1e-6)
    return np.abs(fd - g).max() / np.abs(g).max()


def test_planted_skalak_energy_factor_fails_the_potential_pin(monkeypatch):
    """W halved in the energy only (its derivative untouched)."""
    assert _energy_gradient_mismatch() <= 1e-6
    real = OM.skalak_density

    def planted(F, ct):
        W, dW = real(F, ct)
        return 0.5 * W, dW
    monkeypatch.setattr(OM, "skalak_density", planted)
    assert _energy_gradient_mismatch() > 1e-3


def _volume_term_error():
    base = dict(shear_B=3.0, area_C=40.0, k_bend=2.0)
    ct0 = _small(I.icosahedron, material=I.Material(k_vol=0.0, **base))
    ct1 = _small(I.icosahedron, material=I.Material(k_vol=7.0, **base))
    rng = np.random.default_rng(302)
    x = (ct0.X * 1.05 + 0.05 * rng.normal(size=ct0.X.shape))[None]
    y = ct0.X[None]
    dV = ct1.V0 - O.volume(x, ct1.tri)[0]
    gV = O.volume_gradient(x, ct1.tri)[0]
    expect = 0.5 * 7.0 * dV ** 2 / np.sum(gV * gV)
    got = O.energy(x, y, ct1)[0] - O.energy(x, y, ct0)[0]
    return abs(got - expect) / abs(expect)


def test_planted_volume_projection_step_fails_the_volume_term_pin(monkeypatch):
    """The linearised volume projection moved twice as far (lambda doubled)."""
    assert _volume_term_error() <= 1e-10
    real = OM.volume_projection

    def planted(x, ct):
        p, lam, V = real(x, ct)
        return x + 2.0 * (p - x), lam, V
    monkeypatch.setattr(OM, "volume_projection", planted)
    assert _volume_term_error() > 0.5


def _line_search_steps():
    mat = I.Material(shear_B=0.0, area_C=0.0, k_bend=0.0, k_vol=0.0, membrane="skalak")
    ct = _small(I.icosahedron, material=mat)
    cs = np.array([0.5, 1.5, 3.0, 5.0, 1000.0])
    rng = np.random.default_rng(304)
    N = len(cs)
    y = np.broadcast_to(ct.X, (N, ct.n, 3)) + 0.01 * rng.normal(size=(N, ct.n, 3))
    p = y + 0.2 * rng.normal(size=y.shape)
    w = np.broadcast_to((cs * ct.mass / ct.h ** 2)[:, None], (N, ct.n)).copy()
    x1 = O.line_search_update(ct, y.copy(), y, (p, w))
    return ((x1 - y) / (-cs[:, None, None] * (y - p)))[:, 0, 0]


@pytest.mark.parametrize("name,value", [("ARMIJO_C", -1e-4), ("MAX_HALVINGS", 7)])
def test_planted_line_search_constant_fails_the_step_length_pin(monkeypatch, name, value):
    """The sufficient-decrease test with the constant's sign flipped, or one halving fewer."""
    expect = np.array([1.0, 0.5, 0.25, 0.25, 1.0 / 256])
    assert np.allclose(_line_search_steps(), expect, rtol=1e-9, atol=0)
    monkeypatch.setattr(OM, name, value)
    assert not np.allclose(_line_search_steps(), expect, rtol=1e-9, atol=0)

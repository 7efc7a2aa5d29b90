"""Plain FP64 CPU oracle of the npFEM projective-dynamics time step.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module. The GPU library shares no code with it: it has its own setup
(in C++) and its own kernels (HIP), and neither side imports the other.

What it computes (supplementary material, "Nodal Projective FEM (npFEM)" subsection):
  * implicit Euler, v_{n+1} = (x_{n+1} - x_n)/h  (first displayed equation) and
    F_int(x_{n+1}) + F_ext(x_n) - C v_{n+1} = M (v_{n+1} - v_n)/h (second), with C = 0;
  * the equivalent minimisation of g(x) = 1/(2h^2) ||M^(1/2)(x - y_n)||_F^2 + sum_i E_i(x),
    y_n = x_n + h v_n + h^2 M^-1 F_ext (third displayed equation, C = 0);
  * the quasi-Newton iteration x^{k+1} = x^k - H~ grad g(x^k) with a constant Hessian
    approximation H~ (fourth displayed equation), here H~ = L^-1 where L is the Hessian of the
    quadratic part of g; with projective-dynamics energies this is the local/global iteration.

The paper does not write out the elemental energies E_i (it defers to the npFEM journal
paper). They are read here as projective-dynamics constraint energies
w/2 ||A x - p(x)||^2 with exact projections p:
  * per triangle: strain (singular values clamped to [s_min, s_max]; [1, 1] = polar factor)
    and area (singular values (d, 1/d) nearest to (s1, s2)), weights shear_B * A_t and
    area_C * A_t (Skalak B and C of the parameter table);
  * per interior edge: isometric quadratic bending (cotangent stencil, Bergou et al. 2006 /
    Wardetzky et al. 2007) projected onto its rest norm, weight k_bending;
  * per cell: volume, projected by one linearised step onto V = V0, weight k_volume per vertex;
  * uniform lumped mass m = density * V0 / n (the mass matrix is the lumped total mass,
    interior fluid included, npFEM subsection);
  * optional position-based damping of the velocities (npFEM subsection, after Mueller et al.
    2007): per cell the rigid part of v_n is kept and the rest scaled by 1 - kappa, applied
    to v_n before the prediction (the order of position-based dynamics: damp, then predict);
  * optional Rayleigh damping C = alpha M + beta K (parameter table: alpha_D, beta_D), with K
    the constant stiffness of the strain, area and bending energies (the quadratic part of L
    without the mass and volume terms): M~ = M + h C enters y_n and g(x) as in the
    minimisation form (npFEM subsection), and the quasi-Newton matrix becomes
    M~/h^2 + w_v I + K; alpha in 1/us and beta in us (the solver's time unit);
  * optional Skalak membrane (material `membrane` = "skalak"): the strain and area constraints
    are replaced by the Skalak strain energy per unit rest area
    W = (B/4)(I1^2 + 2 I1 - 2 I2) + (C/4) I2^2, I1 = tr(F^T F) - 2, I2 = det(F^T F) - 1
    (Skalak et al. 1973; B, C of the parameter table); the quasi-Newton direction keeps the
    same prefactored L and the step length comes from a backtracking (Armijo) line search on
    g, per cell;
  * optional collision energies (particle-in-kernel technique, supplementary material): for a
    vertex in contact, (w_i/2) ||x_i - p_i||^2 toward the projection point p_i of the closest
    foreign particle, added to g and its gradient but not to L (the caller supplies p and w,
    and zeroes F_ext at contacting vertices as the technique prescribes);
  * contact detection of the technique (pik_contacts): the colliding neighbour of a vertex is
    the closest vertex of another cell inside the kernel sphere, and its projection point
    lies at a given separation from that neighbour along the neighbour cell's outward vertex
    normal; the packing step (packing_step) is one step with these contacts and no external
    force (main text: cells placed at random and advanced with the fluid switched off);
  * optional capping of the new vertex velocities at v_max (the velocity truncation for the
    stability of the immersed-boundary coupling, Fluid-structure interaction subsection);
Everything is float64, vectorised over the cells of one type (arrays [N][n][3]).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

# ----------------------------------------------------------------------------------------
# Cell-type setup: rest frames, bending stencils, mass and the constant system matrix L.
# ----------------------------------------------------------------------------------------


class CellType:
    """Per-type constants of the step (all float64).

    Attributes
    ----------
    n, m, e : vertices, triangles, interior edges (hinges)
    tri     : int [m][3]
    G       : [m][3][2]  gradient vectors g_a, g_b, g_c of the linear triangle (F = sum_j x_j g_j^T)
    area    : [m]        rest triangle areas A_t
    hinge   : int [e][4] (i, j, k, l): edge (i, j), opposite vertices k and l
    coef    : [e][4]     bending stencil a_e
    rest_norm : [e]      ||sum_q a_e,q X_q|| at rest
    V0, mass, h         rest volume, per-vertex lumped mass, time step
    w_s, w_a, w_b, w_v  constraint weights (shear, area, bending, volume)
    L       : [n][n]     constant system matrix (Hessian of the quadratic part of g)
    """

    def __init__(self, rest_xyz, tri, material, h: float):
        X = np.asarray(rest_xyz, dtype=np.float64)
        tri = np.asarray(tri, dtype=np.int64)
        self.X, self.tri = X, tri
        self.n, self.m = X.shape[0], tri.shape[0]
        self.h = float(h)
        self.w_s = float(material.shear_B)
        self.w_a = float(material.area_C)
        self.w_b = float(material.k_bend)
        self.w_v = float(material.k_vol)
        self.s_min = float(material.strain_min)
        self.s_max = float(material.strain_max)
        self.kappa = float(getattr(material, "pbd_kappa", 0.0))
        self.v_max = float(getattr(material, "v_max", 0.0))
        self.skalak = getattr(material, "membrane", "pd") == "skalak"
        self.alpha = float(getattr(material, "rayleigh_alpha", 0.0))
        self.beta = float(getattr(material, "rayleigh_beta", 0.0))

        self.G, self.area = triangle_rest_frames(X, tri)
        self.hinge, self.coef, self.rest_norm = bending_stencils(X, tri)
        self.e = self.hinge.shape[0]
        self.V0 = float(volume(X[None], tri)[0])
        self.mass = float(material.density) * self.V0 / self.n
        self.L = system_matrix(self)
        self.cho = scipy.linalg.cho_factor(self.L, lower=True)
        self.rayleigh = self.alpha != 0.0 or self.beta != 0.0
        if self.rayleigh:
            # M~ = (1 + h alpha) M + h beta K
            self.K = stiffness_matrix(self)
            self.Mt = (1.0 + self.h * self.alpha) * self.mass * np.eye(self.n) + self.h * self.beta * self.K
            self.cho_Mt = scipy.linalg.cho_factor(self.Mt, lower=True)


def triangle_rest_frames(X, tri):
    """Rest 2D frame per triangle t = (a, b, c).

    e1 = X_b - X_a, e2 = X_c - X_a, t1 = e1/|e1|, t2 = normalise(e2 - (e2.t1) t1);
    D_m = [[|e1|, e2.t1], [0, e2.t2]] holds the rest edges in that frame, and
    F = [x_b - x_a, x_c - x_a] D_m^-1, i.e. g_b = row 0 of D_m^-1, g_c = row 1,
    g_a = -g_b - g_c. Returns G [m][3][2] and rest areas A_t = |e1 x e2|/2.
    """
    a, b, c = X[tri[:, 0]], X[tri[:, 1]], X[tri[:, 2]]
    e1, e2 = b - a, c - a
    l1 = np.linalg.norm(e1, axis=1)
    t1 = e1 / l1[:, None]
    d12 = np.einsum("ij,ij->i", e2, t1)
    perp = e2 - d12[:, None] * t1
    l2 = np.linalg.norm(perp, axis=1)
    Dm = np.zeros((len(tri), 2, 2))
    Dm[:, 0, 0] = l1
    Dm[:, 0, 1] = d12
    Dm[:, 1, 1] = l2
    Bm = np.linalg.inv(Dm)
    G = np.empty((len(tri), 3, 2))
    G[:, 1, :] = Bm[:, 0, :]
    G[:, 2, :] = Bm[:, 1, :]
    G[:, 0, :] = -G[:, 1, :] - G[:, 2, :]
    area = 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    return G, area


def _cot(u, v):
    return np.einsum("ij,ij->i", u, v) / np.linalg.norm(np.cross(u, v), axis=1)


def interior_edges(tri):
    """Hinges (i, j, k, l): (i, j, k) and (j, i, l) are the two triangles of edge {i, j},
    each in its own counter-clockwise order. One hinge per edge of a closed mesh."""
    opp = {}
    for t in tri:
        for r in range(3):
            p, q, o = int(t[r]), int(t[(r + 1) % 3]), int(t[(r + 2) % 3])
            opp[(p, q)] = o
    hinges = []
    for (p, q), o in opp.items():
        if p < q:
            hinges.append((p, q, o, opp[(q, p)]))
    return np.asarray(sorted(hinges), dtype=np.int64)


def bending_stencils(X, tri):
    """Isometric quadratic bending stencil a_e over (i, j, k, l) and its rest norm.

    With e0 = X_j - X_i, e1 = X_k - X_i, e2 = X_l - X_i, e3 = X_k - X_j, e4 = X_l - X_j and
    c_pq = cot of the angle between e_p and e_q (angles at j taken against -e0):
    a_e = sqrt(3/(A0 + A1)) (c03 + c04, c01 + c02, -c01 - c03, -c02 - c04), where A0, A1
    are the areas of triangles (i, j, k) and (j, i, l).
    """
    H = interior_edges(tri)
    i, j, k, l = (X[H[:, q]] for q in range(4))
    e0, e1, e2, e3, e4 = j - i, k - i, l - i, k - j, l - j
    c01, c02 = _cot(e0, e1), _cot(e0, e2)
    c03, c04 = _cot(-e0, e3), _cot(-e0, e4)
    A0 = 0.5 * np.linalg.norm(np.cross(e0, e1), axis=1)
    A1 = 0.5 * np.linalg.norm(np.cross(e0, e2), axis=1)
    s = np.sqrt(3.0 / (A0 + A1))
    coef = s[:, None] * np.stack([c03 + c04, c01 + c02, -c01 - c03, -c02 - c04], axis=1)
    u = np.einsum("eq,eqd->ed", coef, X[H])
    return H, coef, np.linalg.norm(u, axis=1)


def stiffness_matrix(ct: CellType) -> np.ndarray:
    """K = sum_t (w_s + w_a) A_t G_t^T G_t + sum_e w_b a_e a_e^T: the constant stiffness of the
    strain, area and bending energies (the K of Rayleigh damping)."""
    n = ct.n
    K = np.zeros((n, n))
    wt = (ct.w_s + ct.w_a) * ct.area
    for p in range(3):
        for q in range(3):
            np.add.at(K, (ct.tri[:, p], ct.tri[:, q]),
                      wt * np.einsum("tk,tk->t", ct.G[:, p, :], ct.G[:, q, :]))
    for p in range(4):
        for q in range(4):
            np.add.at(K, (ct.hinge[:, p], ct.hinge[:, q]), ct.w_b * ct.coef[:, p] * ct.coef[:, q])
    return K


def system_matrix(ct: CellType) -> np.ndarray:
    """L = (m/h^2 + w_v) I + sum_t (w_s + w_a) A_t G_t^T G_t + sum_e w_b a_e a_e^T.

    It is the Hessian of the quadratic part of g, shared by the three coordinates and by
    every cell of the type. With Rayleigh damping the mass term is M~/h^2:
    L = ((1 + h alpha) m/h^2 + w_v) I + (1 + beta/h) K.
    """
    n = ct.n
    if ct.alpha != 0.0 or ct.beta != 0.0:
        return (np.eye(n) * ((1.0 + ct.h * ct.alpha) * ct.mass / ct.h ** 2 + ct.w_v)
                + (1.0 + ct.beta / ct.h) * stiffness_matrix(ct))
    L = np.eye(n) * (ct.mass / ct.h ** 2 + ct.w_v)
    wt = (ct.w_s + ct.w_a) * ct.area
    for p in range(3):
        for q in range(3):
            np.add.at(L, (ct.tri[:, p], ct.tri[:, q]),
                      wt * np.einsum("tk,tk->t", ct.G[:, p, :], ct.G[:, q, :]))
    for p in range(4):
        for q in range(4):
            np.add.at(L, (ct.hinge[:, p], ct.hinge[:, q]), ct.w_b * ct.coef[:, p] * ct.coef[:, q])
    return L


# ----------------------------------------------------------------------------------------
# Geometry of a deformed state x [N][n][3].
# ----------------------------------------------------------------------------------------


def deformation_gradients(x, ct):
    """F [N][m][3][2] = sum_j x_j g_j^T over the triangle's vertices."""
    return np.einsum("nmjd,mjk->nmdk", x[:, ct.tri], ct.G)


def bending_vectors(x, ct):
    """u [N][e][3] = sum_q a_e,q x_h(q)."""
    return np.einsum("eq,neqd->ned", ct.coef, x[:, ct.hinge])


def volume(x, tri=None):
    """Enclosed volume V = 1/6 sum_t x_a . (x_b x x_c), per cell [N]."""
    if tri is None:
        raise ValueError("tri required")
    a, b, c = x[:, tri[:, 0]], x[:, tri[:, 1]], x[:, tri[:, 2]]
    return np.einsum("nmd,nmd->n", a, np.cross(b, c)) / 6.0


def volume_gradient(x, tri):
    """dV/dx_i [N][n][3] = 1/6 sum over triangles containing i of (cyclic) x_b x x_c."""
    a, b, c = x[:, tri[:, 0]], x[:, tri[:, 1]], x[:, tri[:, 2]]
    g = np.zeros_like(x)
    np.add.at(g, (slice(None), tri[:, 0]), np.cross(b, c) / 6.0)
    np.add.at(g, (slice(None), tri[:, 1]), np.cross(c, a) / 6.0)
    np.add.at(g, (slice(None), tri[:, 2]), np.cross(a, b) / 6.0)
    return g


def surface_area(x, tri):
    a, b, c = x[:, tri[:, 0]], x[:, tri[:, 1]], x[:, tri[:, 2]]
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=-1).sum(axis=1)


# ----------------------------------------------------------------------------------------
# Local step: projections.
# ----------------------------------------------------------------------------------------


def area_root(s1, s2):
    """Singular value d of the nearest area-preserving stretch (d, 1/d) to (s1, s2).

    Stationary points of (t - s1)^2 + (1/t - s2)^2 over t > 0 are the positive roots of
    t^4 - s1 t^3 + s2 t - 1 = 0. All roots come from the companion-matrix eigenvalues
    (as numpy.roots does), the positive real ones are polished by Newton in float64 and the
    one with the smallest objective is returned.
    """
    s1 = np.asarray(s1, dtype=np.float64)
    s2 = np.asarray(s2, dtype=np.float64)
    shape = s1.shape
    s1f, s2f = s1.ravel(), s2.ravel()
    P = s1f.size
    C = np.zeros((P, 4, 4))
    C[:, 0, 0] = s1f
    C[:, 0, 2] = -s2f
    C[:, 0, 3] = 1.0
    C[:, 1, 0] = C[:, 2, 1] = C[:, 3, 2] = 1.0
    r = np.linalg.eigvals(C)
    re = r.real
    ok = (np.abs(r.imag) <= 1e-6 * np.maximum(1.0, np.abs(re))) & (re > 0)
    t = np.where(ok, re, 1.0)
    for _ in range(4):
        f = ((t - s1f[:, None]) * t) * t * t + s2f[:, None] * t - 1.0
        fp = (4.0 * t - 3.0 * s1f[:, None]) * t * t + s2f[:, None]
        t = np.where(ok & (fp != 0), t - f / np.where(fp != 0, fp, 1.0), t)
    obj = (t - s1f[:, None]) ** 2 + (1.0 / t - s2f[:, None]) ** 2
    obj = np.where(ok & (t > 0), obj, np.inf)
    best = np.argmin(obj, axis=1)
    d = t[np.arange(P), best]
    if not np.all(np.isfinite(obj[np.arange(P), best])):
        raise FloatingPointError("area projection found no positive real root")
    return d.reshape(shape)


def triangle_projections(F, ct):
    """(p_strain, p_area), each [N][m][3][2], from the thin SVD F = U diag(s) V^T."""
    U, s, Vh = np.linalg.svd(F, full_matrices=False)
    ss = np.clip(s, ct.s_min, ct.s_max)
    p_s = U @ (ss[..., :, None] * Vh)
    d = area_root(s[..., 0], s[..., 1])
    sa = np.stack([d, 1.0 / d], axis=-1)
    p_a = U @ (sa[..., :, None] * Vh)
    return p_s, p_a


def bending_projection(u, ct):
    """p = r_e u/||u||; when u = 0 the constraint contributes nothing (p = u)."""
    nrm = np.linalg.norm(u, axis=-1, keepdims=True)
    safe = np.where(nrm > 0, nrm, 1.0)
    return np.where(nrm > 0, ct.rest_norm[None, :, None] * u / safe, u)


def volume_projection(x, ct):
    """One linearised step onto V = V0: p = x + lambda grad V, lambda = (V0 - V)/||grad V||^2.

    Returns (p [N][n][3], lambda [N], V [N]).
    """
    V = volume(x, ct.tri)
    gV = volume_gradient(x, ct.tri)
    G2 = np.einsum("nid,nid->n", gV, gV)
    lam = np.where(G2 > 0, (ct.V0 - V) / np.where(G2 > 0, G2, 1.0), 0.0)
    return x + lam[:, None, None] * gV, lam, V


# ----------------------------------------------------------------------------------------
# Objective, gradient, global step.
# ----------------------------------------------------------------------------------------


def _scatter_triangles(ct, M, N):
    """Sum over triangles of M_t g_j into vertex j: M [N][m][3][2] -> [N][n][3]."""
    out = np.zeros((N, ct.n, 3))
    for j in range(3):
        np.add.at(out, (slice(None), ct.tri[:, j]), np.einsum("nmdk,mk->nmd", M, ct.G[:, j, :]))
    return out


def _scatter_hinges(ct, W, N):
    """Sum over hinges of a_e,q W_e into vertex h(q): W [N][e][3] -> [N][n][3]."""
    out = np.zeros((N, ct.n, 3))
    for q in range(4):
        np.add.at(out, (slice(None), ct.hinge[:, q]), ct.coef[None, :, q, None] * W)
    return out


def _mass_term(ct, d):
    """(M~/h^2) d for d [N][n][3]: (m/h^2) d without damping."""
    if not ct.rayleigh:
        return (ct.mass / ct.h ** 2) * d
    return (np.einsum("ij,njd->nid", ct.Mt, d)) / ct.h ** 2


def skalak_density(F, ct):
    """Skalak strain energy per unit rest area W [N][m] and its derivative dW/dF [N][m][3][2]:
    with C = F^T F, I1 = tr C - 2, I2 = det C - 1, W = (B/4)(I1^2 + 2 I1 - 2 I2) + (C/4) I2^2;
    dW/dC = (B/2)(I1 + 1) 1 + (C I2 - B)/2 adj(C) (d det C / dC = adj C), dW/dF = 2 F dW/dC."""
    C = np.einsum("nmdk,nmdl->nmkl", F, F)
    I1 = C[..., 0, 0] + C[..., 1, 1] - 2.0
    I2 = C[..., 0, 0] * C[..., 1, 1] - C[..., 0, 1] * C[..., 1, 0] - 1.0
    B, Cc = ct.w_s, ct.w_a
    W = 0.25 * B * (I1 ** 2 + 2.0 * I1 - 2.0 * I2) + 0.25 * Cc * I2 ** 2
    adj = np.empty_like(C)
    adj[..., 0, 0], adj[..., 1, 1] = C[..., 1, 1], C[..., 0, 0]
    adj[..., 0, 1], adj[..., 1, 0] = -C[..., 0, 1], -C[..., 1, 0]
    dWdC = (0.5 * B * (I1 + 1.0))[..., None, None] * np.eye(2) + (0.5 * (Cc * I2 - B))[..., None, None] * adj
    return W, 2.0 * np.einsum("nmdk,nmkl->nmdl", F, dWdC)


def gradient(x, y, ct, contacts=None):
    """grad g(x) [N][n][3] with projections recomputed at x (local step of the iteration);
    contacts = (p [N][n][3], w [N][n]) adds w (x - p)."""
    N = x.shape[0]
    F = deformation_gradients(x, ct)
    if ct.skalak:
        M = ct.area[None, :, None, None] * skalak_density(F, ct)[1]
    else:
        p_s, p_a = triangle_projections(F, ct)
        M = ct.area[None, :, None, None] * (ct.w_s * (F - p_s) + ct.w_a * (F - p_a))
    u = bending_vectors(x, ct)
    p_b = bending_projection(u, ct)
    p_v, _, _ = volume_projection(x, ct)
    g = _mass_term(ct, x - y)
    g += _scatter_triangles(ct, M, N)
    g += _scatter_hinges(ct, ct.w_b * (u - p_b), N)
    g += ct.w_v * (x - p_v)
    if contacts is not None:
        p_c, w_c = contacts
        g += w_c[..., None] * (x - p_c)
    return g


def pd_rhs(x, y, ct):
    """Projective-dynamics global right-hand side (M/h^2) y + sum_c w_c A_c^T p_c(x)."""
    N = x.shape[0]
    F = deformation_gradients(x, ct)
    p_s, p_a = triangle_projections(F, ct)
    M = ct.area[None, :, None, None] * (ct.w_s * p_s + ct.w_a * p_a)
    u = bending_vectors(x, ct)
    p_b = bending_projection(u, ct)
    p_v, _, _ = volume_projection(x, ct)
    b = _mass_term(ct, y)
    b += _scatter_triangles(ct, M, N)
    b += _scatter_hinges(ct, ct.w_b * p_b, N)
    b += ct.w_v * p_v
    return b


def energy(x, y, ct, contacts=None):
    """g(x) per cell [N] with projections at x (and the contact energies, if any)."""
    F = deformation_gradients(x, ct)
    u = bending_vectors(x, ct)
    p_b = bending_projection(u, ct)
    p_v, _, _ = volume_projection(x, ct)
    e = 0.5 * np.einsum("nid,nid->n", x - y, _mass_term(ct, x - y))
    if ct.skalak:
        e += np.einsum("t,nt->n", ct.area, skalak_density(F, ct)[0])
    else:
        p_s, p_a = triangle_projections(F, ct)
        e += np.einsum("t,ntdk->n", 0.5 * ct.area * ct.w_s, (F - p_s) ** 2)
        e += np.einsum("t,ntdk->n", 0.5 * ct.area * ct.w_a, (F - p_a) ** 2)
    e += 0.5 * ct.w_b * np.einsum("ned,ned->n", u - p_b, u - p_b)
    e += 0.5 * ct.w_v * np.einsum("nid,nid->n", x - p_v, x - p_v)
    if contacts is not None:
        p_c, w_c = contacts
        e += 0.5 * np.einsum("ni,nid,nid->n", w_c, x - p_c, x - p_c)
    return e


def solve(ct, b, method: str = "cholesky"):
    """L^-1 b for b [N][n][3]: the three coordinates of every cell share L."""
    N = b.shape[0]
    B = np.transpose(b, (1, 0, 2)).reshape(ct.n, N * 3)
    if method == "cholesky":
        X = scipy.linalg.cho_solve(ct.cho, B)
    elif method == "dense":
        X = np.linalg.solve(ct.L, B)
    else:
        raise ValueError(method)
    return np.transpose(X.reshape(ct.n, N, 3), (1, 0, 2))


def rigid_velocity_fit(x, v):
    """Centre-of-mass velocity v_cm, angular velocity w and centre x_cm of the rigid motion
    that conserves the linear and angular momentum of the velocity field v at x (equal
    masses): v_cm = mean v, w = I^-1 L with L = sum r x v, I = sum (|r|^2 1 - r r^T),
    r = x - x_cm. x, v: [N][n][3]; returns ([N][3], [N][3], [N][3])."""
    xcm = x.mean(axis=1)
    vcm = v.mean(axis=1)
    r = x - xcm[:, None, :]
    Lm = np.cross(r, v).sum(axis=1)
    rr = np.einsum("nid,nid->n", r, r)
    I = rr[:, None, None] * np.eye(3)[None] - np.einsum("nid,nie->nde", r, r)
    w = np.linalg.solve(I, Lm[:, :, None])[:, :, 0]
    return vcm, w, xcm


def pbd_damp(x, v, kappa: float):
    """Position-based damping of velocities (npFEM subsection; Mueller et al. 2007):
    v <- v + kappa (v_cm + w x r - v), keeping the rigid part of each cell's motion."""
    if kappa == 0.0:
        return v
    vcm, w, xcm = rigid_velocity_fit(x, v)
    r = x - xcm[:, None, :]
    rigid = vcm[:, None, :] + np.cross(w[:, None, :], r)
    return v + kappa * (rigid - v)


def predict(x, v, f, ct):
    """y_n = x_n + h M~^-1 M v_n + h^2 M~^-1 F_ext (third displayed equation; M~ = M without
    Rayleigh damping: y_n = x_n + h v_n + h^2 F_ext / m), with v_n damped first when the type
    has position-based damping."""
    vd = pbd_damp(x, v, ct.kappa)
    if not ct.rayleigh:
        return x + ct.h * vd + (ct.h ** 2 / ct.mass) * f
    rhs = ct.h * ct.mass * vd + ct.h ** 2 * f                                   # [N][n][3]
    N = x.shape[0]
    B = np.transpose(rhs, (1, 0, 2)).reshape(ct.n, N * 3)
    Y = scipy.linalg.cho_solve(ct.cho_Mt, B)
    return x + np.transpose(Y.reshape(ct.n, N, 3), (1, 0, 2))


def step(ct, x, v, f, n_iters: int, form: str = "qn", method: str = "cholesky",
         history: list | None = None, contacts=None):
    """One implicit-Euler step for N cells of one type; x, v, f are [N][n][3] float64.

    The iteration starts at x^0 = y and performs ``n_iters`` quasi-Newton updates
    x^{k+1} = x^k - L^-1 grad g(x^k) (form "qn") or the algebraically identical
    projective-dynamics updates x^{k+1} = L^-1 rhs(x^k) (form "pd"). n_iters = 0 returns
    the prediction. Returns (x_{n+1}, v_{n+1}) with v_{n+1} = (x_{n+1} - x_n)/h, capped at
    the type's v_max when it has one (positions are not changed by the cap). contacts =
    (p [N][n][3], w [N][n]) adds the collision energies (quasi-Newton form only: they enter
    grad g, not L).
    """
    x = np.asarray(x, dtype=np.float64)
    y = predict(x, v, f, ct)
    xk = y.copy()
    if history is not None:
        history.append(xk.copy())
    for _ in range(n_iters):
        if ct.skalak:
            xk = line_search_update(ct, xk, y, contacts, method)
        elif form == "qn":
            xk = xk - solve(ct, gradient(xk, y, ct, contacts), method)
        elif form == "pd":
            if contacts is not None:
                raise ValueError("contacts enter the quasi-Newton form only")
            xk = solve(ct, pd_rhs(xk, y, ct), method)
        else:
            raise ValueError(form)
        if history is not None:
            history.append(xk.copy())
    return xk, cap_velocities((xk - x) / ct.h, ct.v_max)


ARMIJO_C = 1e-4        # sufficient-decrease constant of the line search
MAX_HALVINGS = 8       # step lengths 1, 1/2, ..., 1/256


def line_search_update(ct, x, y, contacts=None, method: str = "cholesky"):
    """One quasi-Newton iteration with a backtracking line search, per cell: direction
    d = -L^-1 grad g(x); the step length a is the first of 1, 1/2, ..., 2^-MAX_HALVINGS with
    g(x + a d) <= g(x) + ARMIJO_C a grad g(x).d (the last one when none qualifies)."""
    gk = gradient(x, y, ct, contacts)
    d = -solve(ct, gk, method)
    e0 = energy(x, y, ct, contacts)
    slope = np.einsum("nid,nid->n", gk, d)
    a = np.ones(x.shape[0])
    done = np.zeros(x.shape[0], dtype=bool)
    for h in range(MAX_HALVINGS + 1):
        et = energy(x + a[:, None, None] * d, y, ct, contacts)
        done |= et <= e0 + ARMIJO_C * a * slope
        if done.all() or h == MAX_HALVINGS:
            break
        a = np.where(done, a, 0.5 * a)
    return x + a[:, None, None] * d


# ----------------------------------------------------------------------------------------
# Boundary filters of the coupling (Fluid-structure interaction subsection): median filter of
# the external forces over each vertex's one ring, and capping of the vertex velocities.
# ----------------------------------------------------------------------------------------


def one_ring_neighbours(tri, n):
    """Sorted neighbour lists (vertices sharing an edge) of every vertex."""
    nb = [set() for _ in range(n)]
    for a, b, c in np.asarray(tri):
        nb[a].update((b, c))
        nb[b].update((a, c))
        nb[c].update((a, b))
    return [sorted(s) for s in nb]


def median_filter_forces(f, ct):
    """Component-wise median of F_ext over each vertex and its one-ring neighbours (the
    median of an even count is the mean of the two middle values). f: [N][n][3]."""
    nbs = one_ring_neighbours(ct.tri, ct.n)
    out = np.empty_like(f)
    for i, nb in enumerate(nbs):
        out[:, i, :] = np.median(f[:, [i] + nb, :], axis=1)
    return out


def cap_velocities(v, v_max: float):
    """Vertex velocities longer than v_max are scaled back to length v_max (direction kept);
    v_max <= 0 leaves them unchanged."""
    if v_max <= 0:
        return v
    s = np.linalg.norm(v, axis=-1, keepdims=True)
    return np.where(s > v_max, v * (v_max / np.maximum(s, 1e-300)), v)


# ----------------------------------------------------------------------------------------
# Batch helpers: SoA [3][V_total] arrays with cells of mixed types.
# ----------------------------------------------------------------------------------------


def step_batch(cell_types: dict, types, offsets, x, v, f, n_iters: int, cells=None,
               contact_p=None, contact_w=None):
    """Advance the listed cells (default: all) of a SoA batch; returns new (x, v) copies.

    cell_types maps type id -> CellType; x, v, f are float64 [3][V_total].
    Cells of the same type are stepped together (they are independent). contact_p [3][V_total]
    and contact_w [V_total] give the collision energies (w = 0: no contact).
    """
    types = np.asarray(types)
    offsets = np.asarray(offsets)
    cells = np.arange(len(types)) if cells is None else np.asarray(cells)
    xo, vo = x.copy(), v.copy()
    for t, ct in cell_types.items():
        sel = cells[types[cells] == t]
        if sel.size == 0:
            continue
        idx = offsets[sel][:, None] + np.arange(ct.n)[None, :]          # [N][n]
        xs = np.transpose(x[:, idx], (1, 2, 0))
        vs = np.transpose(v[:, idx], (1, 2, 0))
        fs = np.transpose(f[:, idx], (1, 2, 0))
        contacts = None
        if contact_w is not None:
            contacts = (np.transpose(contact_p[:, idx], (1, 2, 0)), contact_w[idx])
        xn, vn = step(ct, xs, vs, fs, n_iters, contacts=contacts)
        xo[:, idx] = np.transpose(xn, (2, 0, 1))
        vo[:, idx] = np.transpose(vn, (2, 0, 1))
    return xo, vo


def median_filter_batch(cell_types: dict, types, offsets, f):
    """median_filter_forces of every cell of a SoA batch; returns a new [3][V_total] array."""
    types = np.asarray(types)
    offsets = np.asarray(offsets)
    out = f.copy()
    for t, ct in cell_types.items():
        sel = np.nonzero(types == t)[0]
        if sel.size == 0:
            continue
        idx = offsets[sel][:, None] + np.arange(ct.n)[None, :]
        fs = np.transpose(f[:, idx], (1, 2, 0))
        out[:, idx] = np.transpose(median_filter_forces(fs, ct), (2, 0, 1))
    return out


def cell_volume_area(cell_types: dict, types, offsets, x, cells=None):
    """[n_cells][2] float64 (V, S) of the listed cells at positions x [3][V_total]."""
    types = np.asarray(types)
    offsets = np.asarray(offsets)
    cells = np.arange(len(types)) if cells is None else np.asarray(cells)
    out = np.zeros((len(cells), 2))
    for t, ct in cell_types.items():
        pos = np.nonzero(types[cells] == t)[0]
        if pos.size == 0:
            continue
        idx = offsets[cells[pos]][:, None] + np.arange(ct.n)[None, :]
        xs = np.transpose(x[:, idx], (1, 2, 0))
        out[pos, 0] = volume(xs, ct.tri)
        out[pos, 1] = surface_area(xs, ct.tri)
    return out


# ----------------------------------------------------------------------------------------
# Particle-in-kernel contact detection and the packing step (supplementary material,
# particle-in-kernel technique; main text, near-contact handling and cell packing).
# ----------------------------------------------------------------------------------------


def vertex_normals(x, tri):
    """Unit outward vertex normals of closed meshes x [N][n][3]: for every vertex, the
    normalised sum over its triangles (a, b, c), counter-clockwise seen from outside, of
    (x_b - x_a) x (x_c - x_a) (the area-weighted normal). Float64."""
    tri = np.asarray(tri)
    a, b, c = x[:, tri[:, 0]], x[:, tri[:, 1]], x[:, tri[:, 2]]
    nt = np.cross(b - a, c - a)
    n = np.zeros_like(x, dtype=np.float64)
    for k in range(3):
        np.add.at(n, (slice(None), tri[:, k]), nt)
    return n / np.linalg.norm(n, axis=-1, keepdims=True)


def closest_foreign_vertex(x, cell_of, radius: float, dtype=np.float64, rows=None):
    """The colliding neighbour of the technique: for every vertex i (or the listed rows) of
    x [3][V], the vertex j of another cell (cell_of [V]) with the smallest squared distance
    ((dx dx + dy dy) + dz dz), computed with every operation rounded in `dtype`, among those
    strictly below radius^2 (radius rounded to dtype, squared in dtype); the smallest j among
    equal distances; -1 where no foreign vertex lies inside the kernel.

    Brute force over pairs. For the rows of one cell, the candidates are the other cells'
    vertices inside that cell's bounding box grown by the radius (plus 0.1 %): every vertex
    within the radius of one of the rows lies there, so the result is the full search's."""
    xd = np.asarray(x).astype(dtype)
    x64 = xd.astype(np.float64)
    cell_of = np.asarray(cell_of)
    r = dtype(radius)
    r2 = dtype(r * r)
    V = xd.shape[1]
    rows = np.arange(V) if rows is None else np.asarray(rows)
    out = np.full(len(rows), -1, dtype=np.int64)
    grow = float(radius) * 1.001
    order = np.argsort(x64[0], kind="stable")
    xs = x64[0][order]
    for c in np.unique(cell_of[rows]):
        sel = np.nonzero(cell_of[rows] == c)[0]
        ri = rows[sel]
        lo = x64[:, ri].min(axis=1) - grow
        hi = x64[:, ri].max(axis=1) + grow
        sub = order[np.searchsorted(xs, lo[0], "left"):np.searchsorted(xs, hi[0], "right")]
        keep = ((x64[1][sub] >= lo[1]) & (x64[1][sub] <= hi[1]) & (x64[2][sub] >= lo[2])
                & (x64[2][sub] <= hi[2]) & (cell_of[sub] != c))
        cand = np.sort(sub[keep])                       # ascending: argmin takes the smallest j
        if cand.size == 0:
            continue
        dx = xd[0][cand][None, :] - xd[0][ri][:, None]
        dy = xd[1][cand][None, :] - xd[1][ri][:, None]
        dz = xd[2][cand][None, :] - xd[2][ri][:, None]
        d2 = (dx * dx + dy * dy) + dz * dz
        j = np.argmin(d2, axis=1)                       # first (smallest) j among equal minima
        hit = d2[np.arange(len(ri)), j] < r2
        out[sel] = np.where(hit, cand[j], -1)
    return out


def pik_contacts(cell_types: dict, types, offsets, x, radius: float, separation: float,
                 weight: float, dtype=np.float64, rows=None):
    """Collision inputs of the technique from positions x [3][V_total]: for a vertex i with a
    colliding neighbour j (closest_foreign_vertex), the projection point
    p_i = x_j + separation * n_j (n_j the unit outward vertex normal of j's cell at j) and the
    weight w_i = weight; otherwise p_i = x_i and w_i = 0. Returns (p [3][R], w [R], j [R]) in
    float64 for the listed rows (default: every vertex)."""
    types = np.asarray(types)
    offsets = np.asarray(offsets)
    V = int(offsets[-1])
    cell_of = np.repeat(np.arange(len(types)), np.diff(offsets))
    rows = np.arange(V) if rows is None else np.asarray(rows)
    j = closest_foreign_vertex(x, cell_of, radius, dtype, rows)
    xf = np.asarray(x, dtype=np.float64)
    p = xf[:, rows].copy()
    w = np.zeros(len(rows))
    hit = np.nonzero(j >= 0)[0]
    for k in hit:
        jj = int(j[k])
        c = int(cell_of[jj])
        ct = cell_types[int(types[c])]
        xs = xf[:, offsets[c]:offsets[c + 1]].T[None]
        n = vertex_normals(xs, ct.tri)[0, jj - offsets[c]]
        p[:, k] = xf[:, jj] + separation * n
        w[k] = weight
    return p, w, j


def packing_step(cell_types: dict, types, offsets, x, v, n_iters: int, radius: float,
                 separation: float, weight: float, dtype=np.float64):
    """One step of the cell-packing run (main text: cells placed at random, interpenetrating,
    then advanced with the fluid and the coupling switched off): contacts from the current
    positions, no external force, and the collision energies in the step. Returns
    (x, v, w) with w the contact weights the step used."""
    p, w, _ = pik_contacts(cell_types, types, offsets, x, radius, separation, weight, dtype)
    f = np.zeros_like(np.asarray(x, dtype=np.float64))
    xn, vn = step_batch(cell_types, types, offsets, np.asarray(x, np.float64),
                        np.asarray(v, np.float64), f, n_iters, contact_p=p, contact_w=w)
    return xn, vn, w

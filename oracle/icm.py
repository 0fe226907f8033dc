"""Plain FP64 CPU oracle of one incompressible Inertial Coupling Method step.

TEST INFRASTRUCTURE ONLY. This module is the slow, obviously-correct reference
that the HIP path is compared with. It shares no code with the HIP path, and
only tests, the smoke check and the CPU-baseline leg of the benchmark may
import it. Nothing in the product path routes through it.

It follows the paper (Balboa Usabiaga, Delgado-Buscalioni, Griffith, Donev,
"Inertial coupling method for particles in an incompressible fluctuating
fluid") step by step:

* Sec. III.A: uniform staggered (MAC) grid; discrete J and S built from a
  tensor product of one-dimensional Peskin kernels, S = (dV_f)^-1 J*.
* Sec. III.A.1, Eq. (JS_invariance): kernel moment conditions; the 3-point
  kernel gives dV = 8 dV_f.
* Sec. III.A.2: the split (shifted) three-point kernel, the mean of two
  copies shifted by -s/2 and +s/2 per axis; its dV uses the cell average of
  sum phi^2, whose sum over nodes depends on the blob position.
* Sec. III.B.2: Crank-Nicolson viscosity and the stochastic flux
  Sigma^n = (kT eta / (dV_f dt))^(1/2) (W^n + W^n^T).
* Sec. III.C (Summary of Algorithm), steps 1-9, with the slip-correction
  options of Eqs. (delta_u_nph) and (delta_u_nph_visc).
* Sec. III.D: Helmholtz solve by Fourier diagonalisation, then projection.
* App. A, Eq. (JPS): m~_f = d/(d-1) rho dV.
* App. B.2, Eq. (thermal_drift): thermal drift spread with the kernel
  derivative.
* App. C, Eqs. (dv_tilde_sol), (dv_eq_modified), (u_np1_modified): the
  momentum-conserving inertial velocity correction.
* Sec. III.B.2, Eq. (Adams_Bashforth), and Sec. I.B: the optional advective
  term D.(rho v v^T), time-lagged with the Adams-Bashforth weights 3/2 and
  -1/2.

Array conventions (shared with the GPU only as a documented convention, not
as code): a face field is an array of shape (3, Nz, Ny, Nx), C order, so x is
the fastest index. Cell (i,j,k) has centre ((i+1/2)h, (j+1/2)h, (k+1/2)h);
v_x[k,j,i] sits at (i h, (j+1/2)h, (k+1/2)h), v_y at ((i+1/2)h, j h,
(k+1/2)h) and v_z at ((i+1/2)h, (j+1/2)h, k h). Blob positions are kept
unwrapped; they are wrapped only when indexing the grid.

Readings of points where the paper is silent or ambiguous are listed in the
project's design notes; the ones that change arithmetic are repeated at the
function that implements them.
"""
from dataclasses import dataclass, field, replace
import numpy as np
import scipy.fft as sfft

from . import philox

SLIP_NONE, SLIP_VISCOUS, SLIP_FULL = 0, 1, 2


# --------------------------------------------------------------------------
# One-dimensional Peskin kernels (Sec. III.A.1)
# --------------------------------------------------------------------------
def phi3(r):
    """Three-point kernel: the minimal-support function obeying
    Eq. (JS_invariance): sum phi = 1, first moment 0, sum phi^2 = 1/2.

    Solving those three conditions for the weights of the three nearest nodes
    (taking the root with phi(0) = 2/3) gives the closed form below.
    """
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    a = r <= 0.5
    b = (r > 0.5) & (r <= 1.5)
    out[a] = (1.0 + np.sqrt(1.0 - 3.0 * r[a] ** 2)) / 3.0
    s = 1.0 - r[b]
    out[b] = (5.0 - 3.0 * r[b] - np.sqrt(np.maximum(1.0 - 3.0 * s * s, 0.0))) / 6.0
    return out


def dphi3(r):
    """Derivative of phi3 with respect to its argument."""
    r = np.asarray(r, dtype=np.float64)
    s = np.abs(r)
    sg = np.sign(r)
    out = np.zeros_like(r)
    a = s <= 0.5
    b = (s > 0.5) & (s <= 1.5)
    out[a] = -r[a] / np.sqrt(1.0 - 3.0 * r[a] ** 2)
    t = 1.0 - s[b]
    out[b] = sg[b] * (-0.5 - t / (2.0 * np.sqrt(np.maximum(1.0 - 3.0 * t * t, 1e-300))))
    return out


def phi4(r):
    """Peskin's four-point kernel (named, not printed, in Sec. III.A.2).

    It is the support-4 function with sum phi = 1, sum over even nodes =
    sum over odd nodes = 1/2, zero first moment and sum phi^2 = 3/8.
    """
    r = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(r)
    a = r <= 1.0
    b = (r > 1.0) & (r <= 2.0)
    out[a] = (3.0 - 2.0 * r[a] + np.sqrt(1.0 + 4.0 * r[a] - 4.0 * r[a] ** 2)) / 8.0
    out[b] = (5.0 - 2.0 * r[b] - np.sqrt(np.maximum(-7.0 + 12.0 * r[b] - 4.0 * r[b] ** 2, 0.0))) / 8.0
    return out


def dphi4(r):
    """Derivative of phi4 with respect to its argument."""
    r = np.asarray(r, dtype=np.float64)
    s = np.abs(r)
    sg = np.sign(r)
    out = np.zeros_like(r)
    a = s <= 1.0
    b = (s > 1.0) & (s <= 2.0)
    sa = s[a]
    out[a] = sg[a] * (-2.0 + (4.0 - 8.0 * sa) / (2.0 * np.sqrt(1.0 + 4.0 * sa - 4.0 * sa * sa))) / 8.0
    sb = s[b]
    out[b] = sg[b] * (-2.0 - (12.0 - 8.0 * sb) / (2.0 * np.sqrt(np.maximum(-7.0 + 12.0 * sb - 4.0 * sb * sb, 1e-300)))) / 8.0
    return out


def kernel_fns(kernel):
    if kernel == 3:
        return phi3, dphi3
    if kernel == 4:
        return phi4, dphi4
    raise ValueError("kernel must be 3 or 4")


def stencil_nodes(kernel, x):
    """Nodes touched by a kernel centred at scaled coordinate x.

    x is the blob coordinate in grid units measured from node 0 of the
    component's grid along this axis. Returns integer nodes (unwrapped) and
    the offsets d = x - node, both of shape x.shape + (P,).
    3-point: nodes round(x) + {-1,0,1}; 4-point: floor(x) + {-1,0,1,2}.
    """
    x = np.asarray(x, dtype=np.float64)
    if kernel == 3:
        m0 = np.floor(x + 0.5)
        offs = np.array([-1.0, 0.0, 1.0])
    else:
        m0 = np.floor(x)
        offs = np.array([-1.0, 0.0, 1.0, 2.0])
    nodes = m0[..., None] + offs
    return nodes.astype(np.int64), x[..., None] - nodes


def sum_phi_sq(kernel):
    """Position-independent sum of phi^2 over nodes (third line of
    Eq. (JS_invariance)), evaluated at a node-centred blob."""
    phi, _ = kernel_fns(kernel)
    _, d = stencil_nodes(kernel, np.array(0.0))
    return float(np.sum(phi(d) ** 2))


# --------------------------------------------------------------------------
# Split (shifted) kernels (Sec. III.A.2)
# --------------------------------------------------------------------------
def split_phi3(r, sigma):
    """Split three-point kernel of Sec. III.A.2 along one axis: the mean of
    phi3 shifted by -sigma/2 and by +sigma/2, sigma = s / h (grid units).
    The d-dimensional kernel is the product of these over the axes, which
    is the paper's 2^-d times the product of the shifted sums."""
    r = np.asarray(r, dtype=np.float64)
    return 0.5 * (phi3(r - 0.5 * sigma) + phi3(r + 0.5 * sigma))


def dsplit_phi3(r, sigma):
    """Derivative of split_phi3 with respect to its argument."""
    r = np.asarray(r, dtype=np.float64)
    return 0.5 * (dphi3(r - 0.5 * sigma) + dphi3(r + 0.5 * sigma))


def phi3_autocorrelation(sigma):
    """A(sigma) = integral over t of phi3(t) phi3(t + sigma), by adaptive
    quadrature with the kinks of both factors as break points."""
    from scipy.integrate import quad
    sigma = float(sigma)
    lo, hi = max(-1.5, -1.5 - sigma), min(1.5, 1.5 - sigma)
    if hi <= lo:
        return 0.0
    kinks = [-0.5, 0.5, -0.5 - sigma, 0.5 - sigma, -1.5 - sigma, 1.5 - sigma]
    pts = sorted({b for b in kinks if lo < b < hi})
    f = lambda t: float(phi3(np.array([t]))[0] * phi3(np.array([t + sigma]))[0])
    val, _ = quad(f, lo, hi, points=pts or None, epsabs=1e-14, epsrel=1e-13, limit=200)
    return val


def mean_sum_phi_sq(kernel, sigma=0.0):
    """Sum over nodes of phi^2, averaged over the blob position within a
    cell. For the Peskin kernels it is the constant of Eq. (JS_invariance).
    For the split kernel the sum depends on the position; expanding the
    square of the mean of the two shifted copies, each copy contributes the
    constant 1/2 and the cross term averages to the autocorrelation of phi3
    at lag sigma: (1 + 2 A(sigma)) / 4."""
    if sigma == 0.0:
        return sum_phi_sq(kernel)
    return 0.25 * (1.0 + 2.0 * phi3_autocorrelation(sigma))


def kernel_of(p):
    """(phi, dphi, node layout) of the kernel of p: the split three-point
    kernel runs on the four-node layout floor(x) + {-1, 0, 1, 2}, which holds
    its support |d| < 3/2 + sigma/2 for sigma <= 1."""
    sigma = float(p.kernel_shift)
    if sigma == 0.0:
        phi, dphi = kernel_fns(p.kernel)
        return phi, dphi, p.kernel
    if p.kernel != 3 or not (0.0 < sigma <= 1.0):
        raise ValueError("the split kernel needs kernel 3 and 0 < s/h <= 1")
    return (lambda r: split_phi3(r, sigma)), (lambda r: dsplit_phi3(r, sigma)), 4


# --------------------------------------------------------------------------
# Parameters and state
# --------------------------------------------------------------------------
@dataclass
class Params:
    n: tuple = (32, 32, 32)          # (Nx, Ny, Nz)
    h: float = 1.0
    rho: float = 1.0
    eta: float = 1.0
    kT: float = 0.0
    dt: float = 0.1
    kernel: int = 3
    slip: int = SLIP_VISCOUS
    thermal_drift: bool = True      # active only when kT > 0
    seed: int = 0
    replica: int = 0
    body_force: tuple = (0.0, 0.0, 0.0)
    wca_eps: float = 0.0            # 0 disables the WCA pair force
    wca_sigma: float = 0.0
    spring_k: float = 0.0           # 0 disables the tether spring
    spring_center: tuple = (0.0, 0.0, 0.0)
    advection: bool = False         # include -D.(rho v v^T) in step 2
    kernel_shift: float = 0.0       # s / h of the split three-point kernel
                                    # (Sec. III.A.2); 0: the plain kernel

    @property
    def cell_volume(self):
        return self.h ** 3

    @property
    def blob_volume(self):
        """dV = (J S 1)^-1 = dV_f / (sum phi^2)^3 (Eq. (dV_JS) with the
        discrete S of Sec. III.A.1). With a split kernel, J S 1 depends on
        the blob position; dV then uses its average over the cell."""
        return self.h ** 3 / mean_sum_phi_sq(self.kernel, float(self.kernel_shift)) ** 3

    @property
    def m_f(self):
        """Entrained fluid mass m_f = rho dV (Sec. I.A)."""
        return self.rho * self.blob_volume

    @property
    def mt_f(self):
        """Effective entrained mass m~_f = d/(d-1) rho dV with d = 3
        (App. A, after Eq. (JPS))."""
        return 1.5 * self.m_f

    @property
    def noise_amplitude(self):
        """(kT eta / (dV_f dt))^(1/2), the prefactor of Sigma^n (Sec. III.B.2)."""
        return np.sqrt(self.kT * self.eta / (self.cell_volume * self.dt))


@dataclass
class State:
    v: np.ndarray                     # (3, Nz, Ny, Nx)
    q: np.ndarray                     # (Nb, 3) unwrapped positions
    u: np.ndarray                     # (Nb, 3)
    m_e: np.ndarray                   # (Nb,)
    f_const: np.ndarray               # (Nb, 3)
    lag_c: np.ndarray                 # (Nb, 3) lagged J L dv
    step: int = 0
    adv_prev: np.ndarray = None       # (3, Nz, Ny, Nx) D.(rho v v^T) of the
                                      # previous step; None: no history yet

    def copy(self):
        return State(self.v.copy(), self.q.copy(), self.u.copy(),
                     self.m_e.copy(), self.f_const.copy(), self.lag_c.copy(),
                     self.step, None if self.adv_prev is None else self.adv_prev.copy())


def zero_field(p):
    nx, ny, nz = p.n
    return np.zeros((3, nz, ny, nx))


def new_state(p, q, u=None, m_e=None, f_const=None):
    q = np.array(q, dtype=np.float64).reshape(-1, 3)
    nb = q.shape[0]
    return State(zero_field(p), q,
                 np.zeros((nb, 3)) if u is None else np.array(u, dtype=np.float64).reshape(nb, 3),
                 np.zeros(nb) if m_e is None else np.array(m_e, dtype=np.float64).reshape(nb),
                 np.zeros((nb, 3)) if f_const is None else np.array(f_const, dtype=np.float64).reshape(nb, 3),
                 np.zeros((nb, 3)), 0)


# --------------------------------------------------------------------------
# Interpolation J and spreading S (Sec. III.A.1)
# --------------------------------------------------------------------------
def _component_weights(p, q, alpha, deriv_axis=None):
    """Per-axis nodes and weights for component alpha of a blob at q.

    Along axis beta the alpha-component grid has nodes at (m + o) h with
    o = 0 if beta == alpha else 1/2. If deriv_axis is given, that axis uses
    phi'(d)/h in place of phi(d).
    """
    phi, dphi, layout = kernel_of(p)
    out = []
    for beta in range(3):
        o = 0.0 if beta == alpha else 0.5
        x = q[:, beta] / p.h - o
        nodes, d = stencil_nodes(layout, x)
        if deriv_axis == beta:
            w = dphi(d) / p.h
        else:
            w = phi(d)
        out.append((np.mod(nodes, p.n[beta]), w))
    return out


def interp(p, v, q):
    """J v: sum over the P^3 nodes of phi(dx) phi(dy) phi(dz) v_alpha."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    nb = q.shape[0]
    u = np.zeros((nb, 3))
    for a in range(3):
        (ix, wx), (iy, wy), (iz, wz) = _component_weights(p, q, a)
        w = wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
        vals = v[a][iz[:, :, None, None], iy[:, None, :, None], ix[:, None, None, :]]
        u[:, a] = np.sum(w * vals, axis=(1, 2, 3))
    return u


def spread(p, F, q, deriv=False, out=None):
    """S F: add dV_f^-1 phi(dx) phi(dy) phi(dz) F_alpha to the alpha faces.

    With deriv=True the alpha-axis weight of component alpha is phi'(d_alpha)/h
    (the derivative of the kernel with respect to the blob coordinate),
    which is what the thermal drift of App. B.2 spreads.
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    F = np.asarray(F, dtype=np.float64).reshape(-1, 3)
    if out is None:
        out = zero_field(p)
    inv_dvf = 1.0 / p.cell_volume
    for a in range(3):
        (ix, wx), (iy, wy), (iz, wz) = _component_weights(p, q, a, a if deriv else None)
        w = wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]
        vals = inv_dvf * w * F[:, a][:, None, None, None]
        I = np.broadcast_to(iz[:, :, None, None], vals.shape)
        J = np.broadcast_to(iy[:, None, :, None], vals.shape)
        K = np.broadcast_to(ix[:, None, None, :], vals.shape)
        np.add.at(out[a], (I.ravel(), J.ravel(), K.ravel()), vals.ravel())
    return out


# --------------------------------------------------------------------------
# Staggered finite-difference operators (real space)
# --------------------------------------------------------------------------
# Axis of the (Nz, Ny, Nx) arrays that carries each Cartesian direction.
AX = {0: 2, 1: 1, 2: 0}


def shift(f, beta, s):
    """f evaluated at index +s along Cartesian direction beta (periodic)."""
    return np.roll(f, -s, axis=AX[beta])


def laplacian(p, v):
    """7-point Laplacian applied to each face component separately."""
    out = np.zeros_like(v)
    for a in range(3):
        for b in range(3):
            out[a] += shift(v[a], b, 1) - 2.0 * v[a] + shift(v[a], b, -1)
    return out / p.h ** 2


def divergence(p, v):
    """Cell-centred divergence: (D v)[i] = sum_a (v_a[i+e_a] - v_a[i]) / h."""
    return sum(shift(v[a], a, 1) - v[a] for a in range(3)) / p.h


def gradient(p, s):
    """Face-centred gradient of a cell field: (G s)_a[i] = (s[i] - s[i-e_a]) / h."""
    return np.stack([(s - shift(s, a, -1)) / p.h for a in range(3)])


def curl(p, v):
    """Edge-centred discrete curl of a face field.

    Component c of the result lives on the edge normal to c; e.g. the z
    component at (i h, j h, (k+1/2) h) is
    (v_y[i] - v_y[i-1])/h - (v_x[j] - v_x[j-1])/h.
    The curl of any discrete gradient G s vanishes identically.
    """
    def d(f, b):
        return (f - shift(f, b, -1)) / p.h
    return np.stack([d(v[2], 1) - d(v[1], 2),
                     d(v[0], 2) - d(v[2], 0),
                     d(v[1], 0) - d(v[0], 1)])


def advection(p, v):
    """Advective momentum flux divergence D.(rho v v^T) at the faces.

    The paper takes the skew-adjoint staggered discretisation of its
    fluctuating-hydrodynamics reference without printing it (Sec. I.B). The
    reading used here is the centred conservative (divergence) form of the
    MAC grid: each momentum component a is a flux balance over the control
    volume around its face, with fluxes
      b = a: rho (v_a averaged along a)^2 at the cell centres, and
      b != a: rho (v_b averaged along a) (v_a averaged along b) on the edges
              shared by the a- and b-faces,
    so that component a gains (F_ab[i + 1/2 e_b] - F_ab[i - 1/2 e_b]) / h.
    It conserves momentum for any v and, for discretely divergence-free v
    (where it equals the skew-symmetric form), kinetic energy.
    """
    A = np.zeros_like(v)
    for a in range(3):
        for b in range(3):
            if a == b:
                # centre (i + 1/2) along a; the face i sees centres i +- 1/2
                c = 0.5 * (v[a] + shift(v[a], a, 1))
                F = p.rho * c * c
                A[a] += (F - shift(F, a, -1)) / p.h
            else:
                # edge at (index - 1/2 e_b) relative to the face of a: v_b
                # averaged over the two b-faces at i and i - e_a, v_a over
                # the two a-faces at i and i - e_b
                vb = 0.5 * (v[b] + shift(v[b], a, -1))
                va = 0.5 * (v[a] + shift(v[a], b, -1))
                F = p.rho * vb * va
                A[a] += (shift(F, b, 1) - F) / p.h
    return A


def stochastic_stress_divergence(p, step):
    """s * D_w Sigma-hat with s = (kT eta/(dV_f dt))^(1/2) (Sec. III.B.2).

    W + W^T is realised on the staggered grid with its diagonal at cell
    centres (2 W_aa, variance 4) and its off-diagonal entries on the edges
    (sqrt(2) W_ab, variance 2): the same distribution as W + W^T. Edge
    (i,j,k) of the xy family sits at (i h, j h, (k+1/2) h), of the xz family
    at (i h, (j+1/2) h, k h), of the yz family at ((i+1/2) h, j h, k h).
    """
    nx, ny, nz = p.n
    W = philox.stress_normals(p.n, step, p.seed, p.replica)
    shp = (nz, ny, nx)
    sxx = 2.0 * W["xx"].reshape(shp)
    syy = 2.0 * W["yy"].reshape(shp)
    szz = 2.0 * W["zz"].reshape(shp)
    r2 = np.sqrt(2.0)
    sxy = r2 * W["xy"].reshape(shp)
    sxz = r2 * W["xz"].reshape(shp)
    syz = r2 * W["yz"].reshape(shp)
    X, Y, Z = 0, 1, 2
    dx = (sxx - shift(sxx, X, -1)) + (shift(sxy, Y, 1) - sxy) + (shift(sxz, Z, 1) - sxz)
    dy = (shift(sxy, X, 1) - sxy) + (syy - shift(syy, Y, -1)) + (shift(syz, Z, 1) - syz)
    dz = (shift(sxz, X, 1) - sxz) + (shift(syz, Y, 1) - syz) + (szz - shift(szz, Z, -1))
    return p.noise_amplitude * np.stack([dx, dy, dz]) / p.h


# --------------------------------------------------------------------------
# Fourier symbols, projection and Helmholtz solve (Sec. II.C, Sec. III.D)
# --------------------------------------------------------------------------
def symbols(p):
    """Discrete divergence and gradient symbols on the rfftn grid.

    With the forward transform V_m = sum_i v_i exp(-2 pi i m i / N), a unit
    shift i -> i+1 multiplies by exp(i theta), theta = 2 pi m / N, so
    D-hat = (e^{i theta} - 1)/h and G-hat = (1 - e^{-i theta})/h. Their
    product summed over axes is the Laplacian symbol
    L-hat = -sum (4/h^2) sin^2(theta/2). Returns (Dhat, Ghat, Lhat), where
    Dhat and Ghat are lists of three arrays broadcastable to (Nz, Ny, Nx/2+1).
    """
    nx, ny, nz = p.n
    th = [2.0 * np.pi * np.arange(nx // 2 + 1) / nx,
          2.0 * np.pi * np.arange(ny) / ny,
          2.0 * np.pi * np.arange(nz) / nz]
    shapes = [(1, 1, -1), (1, -1, 1), (-1, 1, 1)]
    D = [((np.exp(1j * t) - 1.0) / p.h).reshape(s) for t, s in zip(th, shapes)]
    G = [((1.0 - np.exp(-1j * t)) / p.h).reshape(s) for t, s in zip(th, shapes)]
    L = sum(D[a] * G[a] for a in range(3)).real
    return D, G, L


def fft_field(v):
    return sfft.rfftn(v, axes=(1, 2, 3))


def ifft_field(p, vh):
    nx, ny, nz = p.n
    return sfft.irfftn(vh, s=(nz, ny, nx), axes=(1, 2, 3))


def project_hat(p, vh):
    """Apply P-hat = I - G-hat D-hat^T / L-hat per mode (P-hat(0) = I)."""
    D, G, L = symbols(p)
    div = sum(D[a] * vh[a] for a in range(3))
    Ls = np.where(L == 0.0, 1.0, L)
    coef = np.where(L == 0.0, 0.0, div / Ls)
    return np.stack([vh[a] - G[a] * coef for a in range(3)])


def project(p, v):
    return ifft_field(p, project_hat(p, fft_field(v)))


def helmholtz_project(p, rhs, a, b):
    """Solve (a - b L) w + G pi = rhs, D w = 0 by Fourier diagonalisation of L
    followed by projection (Sec. III.D): w-hat = P-hat rhs-hat / (a - b L-hat)."""
    _, _, L = symbols(p)
    wh = fft_field(rhs) / (a - b * L)
    return ifft_field(p, project_hat(p, wh))


# --------------------------------------------------------------------------
# Forces on the blobs (evaluated at the midpoint, Sec. III.C step 1)
# --------------------------------------------------------------------------
def wca_forces(p, q):
    """Pair forces of the WCA potential of Sec. IV.A, Eq. (WCA), with minimum
    image in the periodic box; each unordered pair counted once."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    nb = q.shape[0]
    F = np.zeros((nb, 3))
    if p.wca_eps == 0.0 or nb < 2:
        return F
    L = np.array(p.n, dtype=np.float64) * p.h
    rc = 2.0 ** (1.0 / 6.0) * p.wca_sigma
    chunk = 512
    for s in range(0, nb, chunk):
        d = q[s:s + chunk, None, :] - q[None, :, :]
        d -= L * np.round(d / L)
        r2 = np.sum(d * d, axis=2)
        mask = (r2 < rc * rc) & (r2 > 0.0)
        r2s = np.where(mask, r2, 1.0)
        sr6 = (p.wca_sigma ** 2 / r2s) ** 3
        # -dV/dr / r = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2
        fmag = np.where(mask, 24.0 * p.wca_eps * (2.0 * sr6 * sr6 - sr6) / r2s, 0.0)
        F[s:s + chunk] += np.sum(fmag[:, :, None] * d, axis=1)
    return F


def forces(p, q, f_const):
    """Constant + tether spring -k (q - q_c) (unwrapped) + WCA pairs."""
    F = np.array(f_const, dtype=np.float64).reshape(-1, 3).copy()
    if p.spring_k != 0.0:
        F -= p.spring_k * (q - np.asarray(p.spring_center))
    F += wca_forces(p, q)
    return F


# --------------------------------------------------------------------------
# The time step (Sec. III.C, steps 1-9)
# --------------------------------------------------------------------------
def thermal_drift_coef(p, m_e):
    """kT m~_f / m~ per blob (App. B.2, Eq. (thermal_drift))."""
    if p.kT == 0.0 or not p.thermal_drift:
        return None
    return p.kT * p.mt_f / (m_e + p.mt_f)


def slip_correction(p, lag_c, Jn_vn, Jh_vn):
    """The slip velocity delta-u^{n+1/2} of Sec. III.C step 4.

    FULL, Eq. (delta_u_nph): (J^{n+1/2} - J^n) v^n plus the viscous term;
    VISCOUS, Eq. (delta_u_nph_visc): the viscous term alone,
    (nu dt / 2) J^{n-1/2} L dv^{n-1/2} with nu = eta / rho, where lag_c holds
    J^{n-1/2} L dv^{n-1/2} from the previous step; NONE: zero.
    """
    du = np.zeros_like(np.asarray(lag_c, dtype=np.float64))
    if p.slip == SLIP_FULL:
        du += Jh_vn - Jn_vn
    if p.slip in (SLIP_VISCOUS, SLIP_FULL):
        du += 0.5 * (p.eta / p.rho) * p.dt * lag_c
    return du


def lagged_viscous_term(p, dv, q_h):
    """J^{n+1/2} L dv^{n+1/2}: the term of Eq. (Florens_trick) that App. C
    lags to the next step's slip correction (7-point Laplacian, then J)."""
    return interp(p, laplacian(p, dv), q_h)


def step(p, st, trace=None):
    """Advance one time step. Returns a new State (the input is untouched).

    If trace is a dict, the step stores its intermediate quantities there
    under the paper's names (rhs, v_tilde, du, dp, dv_tilde, g, dv), so that
    tests can check each against what the paper fixes for it.

    Steps follow Sec. III.C. Readings applied here:
    * m_e = 0 blobs report u^{n+1} = J^{n+1/2} v^{n+1} (the m_e -> 0 limit of
      Eq. (update_u)); with m_e = 0 everywhere steps 4-8 are skipped.
    * the lagged viscous slip term c = J^{n-1/2} L dv^{n-1/2} is zero before
      the first step that ran steps 4-8.
    * the multi-blob inverse of rho_eff uses each blob's own coefficient
      m~_f / (rho m~_i) (App. A, Eq. (rho_eff_inv_approx)).
    """
    st = st.copy()
    q_n, v_n = st.q, st.v
    dt, rho, eta = p.dt, p.rho, p.eta
    nb = q_n.shape[0]

    # Step 1: midpoint predictor and forces there.
    Jn_vn = interp(p, v_n, q_n) if nb else np.zeros((0, 3))
    q_h = q_n + 0.5 * dt * Jn_vn
    F = forces(p, q_h, st.f_const) if nb else np.zeros((0, 3))

    # Step 2: unperturbed fluid solve, Eq. (provisional_step-1):
    # (rho/dt - eta/2 L) v~ + G pi~ = rhs. The advective term is optional
    # (off by default); with it, rhs carries -(3/2 A^n - 1/2 A^{n-1}),
    # Eq. (Adams_Bashforth), and the first step with no history uses A^n
    # alone (forward Euler).
    rhs = (rho / dt) * v_n + 0.5 * eta * laplacian(p, v_n)
    adv_new = None
    if p.advection:
        adv_new = advection(p, v_n)
        prev = adv_new if st.adv_prev is None else st.adv_prev
        rhs -= 1.5 * adv_new - 0.5 * prev
    if p.kT > 0.0:
        rhs += stochastic_stress_divergence(p, st.step)
    rhs += np.asarray(p.body_force, dtype=np.float64).reshape(3, 1, 1, 1)
    if nb:
        spread(p, F, q_h, out=rhs)
        coef = thermal_drift_coef(p, st.m_e)
        if coef is not None:
            spread(p, coef[:, None] * np.ones((nb, 3)), q_h, deriv=True, out=rhs)
    v_t = helmholtz_project(p, rhs, rho / dt, 0.5 * eta)
    if trace is not None:
        trace["rhs"] = rhs.copy()
        trace["v_tilde"] = v_t.copy()
        trace["q_half"] = q_h.copy()
        trace["F"] = F.copy()

    Jh_vn = interp(p, v_n, q_h) if nb else np.zeros((0, 3))
    inertial = nb > 0 and np.any(st.m_e != 0.0)
    u_new = st.u.copy()
    lag_new = np.zeros((nb, 3))
    if inertial:
        m_e = st.m_e
        # Step 4: slip correction and excess-momentum change.
        du = slip_correction(p, st.lag_c, Jn_vn, Jh_vn)
        Jh_vt = interp(p, v_t, q_h)
        dp = m_e[:, None] * (st.u - Jh_vt - du)
        # Step 5: dv~ = m~_f / (rho m~) P S dp, Eq. (dv_tilde_sol).
        c5 = p.mt_f / (rho * (p.mt_f + m_e))
        dvt = project(p, spread(p, c5[:, None] * dp, q_h))
        g = interp(p, dvt, q_h)
        # Step 6: (rho - dt/2 eta L) dv + dt G dpi = S (dp - m_e J dv~),
        # Eq. (dv_eq_modified).
        dv = helmholtz_project(p, spread(p, dp - m_e[:, None] * g, q_h), rho, 0.5 * dt * eta)
        # Step 7.
        v_new = v_t + dv
        # Step 8, Eq. (update_u) / (u_np1_modified).
        u_new = Jh_vt + g + du
        lag_new = lagged_viscous_term(p, dv, q_h)
        if trace is not None:
            trace.update(du=du, dp=dp, dv_tilde=dvt, g=g, dv=dv)
    else:
        v_new = v_t

    # Step 9: position update, Eq. (update_q).
    if nb:
        Jh_vnew = interp(p, v_new, q_h)
        q_new = q_n + 0.5 * dt * (Jh_vnew + Jh_vn)
        zero_me = st.m_e == 0.0
        u_new[zero_me] = Jh_vnew[zero_me]
    else:
        q_new = q_n
    return State(v_new, q_new, u_new, st.m_e.copy(), st.f_const.copy(),
                 lag_new, st.step + 1, adv_new)


def run(p, st, n_steps):
    for _ in range(n_steps):
        st = step(p, st)
    return st


# --------------------------------------------------------------------------
# Initial conditions
# --------------------------------------------------------------------------
def kick_field(p, q, u0, m_e):
    """Fluid velocity that gives each blob the impulse m~_f u0 at t = 0:
    v^0 = P S (m~_f u0) / rho, so J v^0 = u0 up to the translational
    invariance error of J P S (Sec. III.A.2). Same operator as step 5 with
    dp = m~ u0 and coefficient m~_f/(rho m~)."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    u0 = np.asarray(u0, dtype=np.float64).reshape(-1, 3)
    return project(p, spread(p, (p.mt_f / p.rho) * u0, q))


def equilibrium_field(p):
    """A sample of the discrete Gibbs-Boltzmann distribution of the fluid:
    every face value N(0, kT/(rho dV_f)) from Philox block 3, then projected,
    so the covariance is (kT/(rho dV_f)) P (Sec. II.F with no blobs)."""
    nx, ny, nz = p.n
    a, b, c = philox.equilibrium_normals(nx * ny * nz, p.seed, p.replica)
    sd = np.sqrt(p.kT / (p.rho * p.cell_volume))
    w = sd * np.stack([a, b, c]).reshape(3, nz, ny, nx)
    return project(p, w)


# --------------------------------------------------------------------------
# Diagnostics (FP64)
# --------------------------------------------------------------------------
def momentum(p, st):
    """Total momentum P = rho dV_f sum v + sum m_e u (Sec. II, after
    Eq. (no_slip); the cell volume enters as in the footnote of Sec. III.A.1)."""
    Pf = p.rho * p.cell_volume * st.v.sum(axis=(1, 2, 3))
    Pb = (st.m_e[:, None] * st.u).sum(axis=0) if st.q.shape[0] else 0.0
    return Pf + Pb


def kinetic_energy(p, st):
    ke_f = 0.5 * p.rho * p.cell_volume * float(np.sum(st.v ** 2))
    ke_b = 0.5 * float(np.sum(st.m_e[:, None] * st.u ** 2)) if st.q.shape[0] else 0.0
    return ke_f, ke_b


def advective_cfl(p, st):
    """The advective CFL number alpha = V dt / dx of Eq. (alpha_beta), with V
    the largest magnitude of any face velocity or blob velocity component
    (the speed at which something crosses a cell along one axis)."""
    V = float(np.max(np.abs(st.v))) if st.v.size else 0.0
    if st.u.size:
        V = max(V, float(np.max(np.abs(st.u))))
    return V * p.dt / p.h


def max_divergence(p, v):
    """max |D v| h / max |v| (0 for a zero field)."""
    vm = float(np.max(np.abs(v)))
    if vm == 0.0:
        return 0.0
    return float(np.max(np.abs(divergence(p, v)))) * p.h / vm


def jps_matrix(p, q):
    """The 3x3 matrix J P S for one blob at q (Sec. III.A.2)."""
    M = np.zeros((3, 3))
    for b in range(3):
        F = np.zeros((1, 3))
        F[0, b] = 1.0
        M[:, b] = interp(p, project(p, spread(p, F, q)), q)[0]
    return M


def mobility_matrix(p, q):
    """Steady Stokes mobility -J L^-1 S of Sec. III.A.2 for one blob, with the
    k = 0 mode removed (zero mean flow in the periodic box)."""
    D, G, L = symbols(p)
    M = np.zeros((3, 3))
    Ls = np.where(L == 0.0, 1.0, L)
    for b in range(3):
        F = np.zeros((1, 3))
        F[0, b] = 1.0
        fh = project_hat(p, fft_field(spread(p, F, q)))
        vh = np.where(L == 0.0, 0.0, -fh / (p.eta * Ls))
        M[:, b] = interp(p, ifft_field(p, vh), q)[0]
    return M

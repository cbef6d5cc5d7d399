"""Lattice operators of the oracle (plain NumPy, complex128).

Full-lattice fields are arrays of shape (T, Lz, Ly, Lx, ...).  A doublet
spinor is (T, Lz, Ly, Lx, 2, 4, 3) = [flavour][spin][colour]; a gauge field is
(T, Lz, Ly, Lx, 4, 3, 3) = [mu][row][col].  Direction mu=0 is time (axis 0),
mu=1 is x (axis 3), mu=2 is y (axis 2), mu=3 is z (axis 1).

Paper references: section 2 (Wilson twisted mass fermions), equations
eq:non-degenerate, eq:D(mu), eq:Wilson, eq:g5tau1-hermiticity and the even-odd
reduction paragraph.

Readings where the paper is silent (listed in the design notes as well):
* the site term of eq:Wilson is a = m + 4 = 1/(2 kappa); the clover term is off
  unless c_sw is given (oracle/clover.py holds its reading of Q_mu_nu);
* chiral gamma basis gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]],
  which gives gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1,1,-1,-1) as the
  paper states;
* periodic boundaries; optional antiperiodic time (sign on links crossing t=T-1 -> 0);
* the even-odd operator keeps the odd sites: S = A - 1/4 H_oe A^-1 H_eo and
  Q = (Gamma5 x tau1) S, which is Hermitian.
"""
from __future__ import annotations

import numpy as np

MU_AXIS = (0, 3, 2, 1)  # lattice axis of direction mu

_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
_SIG = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def gamma_matrices():
    """Chiral-basis Dirac matrices gamma_0..gamma_3 and gamma_5 (section 2)."""
    g0 = np.block([[_Z2, -_I2], [-_I2, _Z2]])
    gs = [g0] + [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _SIG]
    g5 = gs[0] @ gs[1] @ gs[2] @ gs[3]
    return np.array(gs), g5


GAMMA, GAMMA5 = gamma_matrices()
TAU1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
TAU3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


class Lattice:
    """Geometry plus gauge field; dims = (T, Lz, Ly, Lx), all even."""

    def __init__(self, dims, U_canonical=None, antiperiodic_t=False):
        self.dims = tuple(int(d) for d in dims)
        T, Z, Y, X = self.dims
        self.V = T * Z * Y * X
        self.antiperiodic_t = bool(antiperiodic_t)
        t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
        self.parity = (t + z + y + x) % 2
        flat = self.parity.reshape(-1)
        self.odd_sites = np.nonzero(flat == 1)[0]
        self.even_sites = np.nonzero(flat == 0)[0]
        if U_canonical is not None:
            self.U = np.asarray(U_canonical, dtype=np.complex128).reshape(T, Z, Y, X, 4, 3, 3)
        else:
            self.U = None

    # -- field embeddings ---------------------------------------------------
    def full_zeros(self, inner=(2, 4, 3)):
        return np.zeros(self.dims + tuple(inner), dtype=np.complex128)

    def odd_to_full(self, v_odd):
        """(V/2, ...) odd-site vector -> full lattice with zeros on even sites."""
        inner = v_odd.shape[1:]
        f = np.zeros((self.V,) + inner, dtype=np.complex128)
        f[self.odd_sites] = v_odd
        return f.reshape(self.dims + inner)

    def even_to_full(self, v_even):
        inner = v_even.shape[1:]
        f = np.zeros((self.V,) + inner, dtype=np.complex128)
        f[self.even_sites] = v_even
        return f.reshape(self.dims + inner)

    def take_odd(self, f):
        inner = f.shape[4:]
        return f.reshape((self.V,) + inner)[self.odd_sites]

    def take_even(self, f):
        inner = f.shape[4:]
        return f.reshape((self.V,) + inner)[self.even_sites]

    # -- shifts ----------------------------------------------------------------
    def _fwd(self, f, mu):
        """f(x + mu_hat), with the antiperiodic sign when crossing t=T-1 -> 0."""
        g = np.roll(f, -1, axis=MU_AXIS[mu])
        if mu == 0 and self.antiperiodic_t:
            g = g.copy()
            g[-1] *= -1
        return g

    def _bwd(self, f, mu):
        """f(x - mu_hat), with the antiperiodic sign when crossing t=0 -> T-1."""
        g = np.roll(f, 1, axis=MU_AXIS[mu])
        if mu == 0 and self.antiperiodic_t:
            g = g.copy()
            g[0] *= -1
        return g

    # -- operators ---------------------------------------------------------------
    def hop(self, psi):
        """Wilson hopping sum of eq:Wilson acting on each flavour:

        (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
                          + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu).
        psi has shape dims + (nf, 4, 3).
        """
        out = np.zeros_like(psi)
        eye4 = np.eye(4, dtype=np.complex128)
        for mu in range(4):
            Umu = self.U[..., mu, :, :]
            fwd = self._fwd(psi, mu)
            t = np.einsum("...ab,...fsb->...fsa", Umu, fwd)
            out += np.einsum("st,...ftc->...fsc", eye4 - GAMMA[mu], t)
            # U_mu(x - mu); the antiperiodic sign is carried by psi's shift only
            Ub = np.roll(Umu, 1, axis=MU_AXIS[mu])
            bwd = self._bwd(psi, mu)
            t = np.einsum("...ba,...fsb->...fsa", Ub.conj(), bwd)
            out += np.einsum("st,...ftc->...fsc", eye4 + GAMMA[mu], t)
        return out

    def hop_flavour(self, psi1):
        """Hopping sum on a single-flavour field (dims + (4, 3))."""
        return self.hop(psi1[..., None, :, :])[..., 0, :, :]


class NDOperator:
    """Non-degenerate twisted-mass doublet, eq:non-degenerate:

    D_ND = D_W x I_2 + i mubar (Gamma5 x tau3) - epsbar (I x tau1),
    D_W  = a - H/2 with a = 1/(2 kappa)     (eq:Wilson with m + 4 = a, c_sw = 0).
    """

    def __init__(self, lat: Lattice, kappa, mubar, epsbar, csw=0.0):
        self.lat = lat
        self.a = 1.0 / (2.0 * kappa)
        self.mubar = float(mubar)
        self.epsbar = float(epsbar)
        self.csw = float(csw)
        # 8x8 site block over (flavour, spin) in kron(flavour, spin) order.
        self.A_block = (self.a * np.eye(8) + 1j * self.mubar * np.kron(TAU3, GAMMA5)
                        - self.epsbar * np.kron(TAU1, np.eye(4)))
        den = self.a ** 2 + self.mubar ** 2 - self.epsbar ** 2
        if den == 0:
            raise ValueError("a^2 + mubar^2 - epsbar^2 must be nonzero")
        # Closed form: gamma5 tau3 and tau1 anticommute, so
        # A^-1 = (a - i mubar g5 tau3 + epsbar tau1) / (a^2 + mubar^2 - epsbar^2).
        self.Ainv_block = (self.a * np.eye(8) - 1j * self.mubar * np.kron(TAU3, GAMMA5)
                           + self.epsbar * np.kron(TAU1, np.eye(4))) / den
        self.G5T1_block = np.kron(TAU1, GAMMA5)
        if self.csw != 0.0:
            # with the clover term of eq:Wilson the site term varies by site: the 24x24 matrix
            # (a + C(x)) x I_2 + i mubar Gamma5 x tau3 - epsbar tau1 over (flavour, spin,
            # colour), inverted numerically on every site
            from .clover import clover_term
            C = clover_term(lat.U, self.csw).reshape(lat.V, 12, 12)
            self.C_site = C
            twist = np.kron(1j * self.mubar * np.kron(TAU3, GAMMA5) - self.epsbar * np.kron(TAU1, np.eye(4)),
                            np.eye(3))
            self.A_site = np.einsum("fg,vij->vfigj", np.eye(2), self.a * np.eye(12) + C).reshape(lat.V, 24, 24)
            self.A_site = self.A_site + twist
            self.Ainv_site = np.linalg.inv(self.A_site)

    # site-local (flavour, spin) blocks acting on [..., f, s, c]
    @staticmethod
    def _site(block8, psi):
        sh = psi.shape
        v = psi.reshape(sh[:-3] + (8, 3))
        return np.einsum("ij,...jc->...ic", block8, v).reshape(sh)

    @staticmethod
    def _per_site(mats, psi):
        sh = psi.shape
        v = psi.reshape(mats.shape[0], 24)
        return np.einsum("vij,vj->vi", mats, v).reshape(sh)

    def A(self, psi):
        """Site term on a full-lattice doublet (dims + (2, 4, 3))."""
        if self.csw == 0.0:
            return self._site(self.A_block, psi)
        return self._per_site(self.A_site, psi)

    def A_odd(self, v_odd):
        if self.csw == 0.0:
            return self._site(self.A_block, v_odd)
        return self._per_site(self.A_site[self.lat.odd_sites], v_odd)

    def Ainv(self, psi):
        """Inverse site term on a full-lattice doublet."""
        if self.csw == 0.0:
            return self._site(self.Ainv_block, psi)
        return self._per_site(self.Ainv_site, psi)

    def Ainv_even(self, v_even):
        if self.csw == 0.0:
            return self._site(self.Ainv_block, v_even)
        return self._per_site(self.Ainv_site[self.lat.even_sites], v_even)

    def g5t1(self, psi):
        return self._site(self.G5T1_block, psi)

    def D_full(self, psi, odd_shift=0.0):
        """D_ND psi on the full lattice; with odd_shift = +-m this is
        D'_+- = D_ND +- i m (Gamma5 x tau1) P_odd (odd-site shift term)."""
        out = self.A(psi) - 0.5 * self.lat.hop(psi)
        if odd_shift != 0.0:
            odd = (self.lat.parity == 1)[..., None, None, None]
            out = out + 1j * odd_shift * np.where(odd, self.g5t1(psi), 0)
        return out

    # even-odd pieces on half vectors of shape (V/2, 2, 4, 3)
    def H_eo(self, v_odd):
        return self.lat.take_even(self.lat.hop(self.lat.odd_to_full(v_odd)))

    def H_oe(self, v_even):
        return self.lat.take_odd(self.lat.hop(self.lat.even_to_full(v_even)))

    def S_hat(self, v_odd):
        """Odd-site Schur complement S = A - 1/4 H_oe A^-1 H_eo (even-odd reduction, section 2)."""
        t = self.Ainv_even(self.H_eo(v_odd))
        return self.A_odd(v_odd) - 0.25 * self.H_oe(t)

    def Q_hat(self, v_odd):
        """Q = (Gamma5 x tau1) S, Hermitian by eq:g5tau1-hermiticity."""
        return self.g5t1(self.S_hat(v_odd))

    def Q_hat2(self, v_odd, sigma=0.0):
        return self.Q_hat(self.Q_hat(v_odd)) + sigma * v_odd

    def S_shift(self, v_odd, m):
        """(S +- i m Gamma5 tau1) v: Gamma5 tau1 times this is Q +- i m."""
        return self.S_hat(v_odd) + 1j * m * self.g5t1(v_odd)


def norm2(v) -> float:
    return float(np.vdot(v, v).real)


def rel_residual(op: NDOperator, x, b, sigma) -> float:
    """||b - (Q^2 + sigma) x|| / ||b|| in FP64."""
    r = b - op.Q_hat2(x, sigma)
    return float(np.sqrt(norm2(r) / norm2(b)))

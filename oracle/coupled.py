"""Algorithm 1, Stage 2: explicit time stepping of the coupled subdomain ROMs.

Per subdomain the ROM in S-fraction coordinates reads (eq. "GammaU" in the time
domain, with flux input g on the boundary layer)

    Gamma-hat^{-1} U_tt = -D^T Gamma D U + Gamma-hat^{-1} s f(t) + E_1 g,

i.e. with layer fluxes phi_j = Gamma_j (U_{j+1} - U_j), U_{k+1} = 0, phi_0 = 0:

    U_j,tt = Gamma-hat_j (phi_j - phi_{j-1}) + s_j f        j = 2..k  (eq. "intrtstep")
    U_1,tt = Gamma-hat_1 (phi_1 + g) + s_1 f.

Continuity of U_1 and flux balance g^alpha + g^beta = 0 on a shared boundary
(eq. "mass") give, for a diagonal Gamma-hat_1 with entries H (eq. "bdrytstep"),

    U_f,tt = C_f ( sum_sides [phi_1]_f + f sum_sides H^{-1} [s_1]_f ),
    C_f = ( sum_sides H^{-1} )^{-1},

one equation per shared unknown ("port"); an outer face has one side and zero
flux (conservative Neumann reading of the outer boundary).  The right-hand
sides are evaluated at the current step (end of the Stage 2 section) and the
integrator is leapfrog, U^{n+1} = 2U^n - U^{n-1} + dt^2 a(U^n, t_n).

``CoupledSystem.accel`` follows steps 2.1-2.3 literally (exchange of face rows
of phi_1, interior update, boundary update).  ``CoupledSystem.assemble`` writes
the same scheme as one global mass/stiffness pair (M, K) for the energy and
CFL checks.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .rom import SubdomainROM
from .subdomains import Subdomain, owner_subdomain, port_table


class CoupledSystem:
    def __init__(self, subs: List[Subdomain], roms: List[SubdomainROM],
                 src_ijk: Sequence = (), rec_ijk: Sequence = (), diag_tol: float = 1e-10):
        self.subs = subs
        self.roms = roms
        self.n_ports, self.port_ids = port_table(subs)
        # Face masses: Gamma-hat_1 must be diagonal for the decoupled scheme (eq. "bdrytstep").
        self.H = []
        inv_sum = np.zeros(self.n_ports)
        for sd, rom in zip(subs, roms):
            gh1 = rom.sf.gamma_hat[0]
            off = gh1 - np.diag(np.diag(gh1))
            if np.abs(off).max() > diag_tol * np.abs(np.diag(gh1)).max():
                raise ValueError(f"subdomain {sd.index}: Gamma-hat_1 is not diagonal")
            H = np.diag(gh1).copy()
            self.H.append(H)
            np.add.at(inv_sum, self.port_ids[sd.index], 1.0 / H)
        self.C = 1.0 / inv_sum
        # Sources: strictly interior to one subdomain.
        self.sources = []
        for s in np.asarray(src_ijk, dtype=np.int64).reshape(-1, 3):
            a = owner_subdomain(subs, s, strict=True)
            if a < 0:
                raise ValueError(f"source {tuple(s)} is not interior to a subdomain")
            sd = subs[a]
            vec = roms[a].source_vector(sd, sd.local_index(s))
            w = np.zeros(self.n_ports)
            np.add.at(w, self.port_ids[a], vec[0] / self.H[a])
            self.sources.append((a, vec, w))
        # Receivers: reconstructed from the lowest-index subdomain whose box holds them.
        self.receivers = []
        for r in np.asarray(rec_ijk, dtype=np.int64).reshape(-1, 3):
            a = owner_subdomain(subs, r)
            if a < 0:
                raise ValueError(f"receiver {tuple(r)} outside the domain")
            sd = subs[a]
            self.receivers.append((a, roms[a].receiver_row(sd, sd.local_index(r))))

    # ------------------------------------------------------------------ Stage 2 steps
    def fluxes(self, U: List[np.ndarray]) -> List[np.ndarray]:
        """phi_j = Gamma_j (U_{j+1} - U_j), j = 1..k, with U_{k+1} = 0."""
        out = []
        for rom, Ua in zip(self.roms, U):
            dU = np.vstack([Ua[1:], np.zeros((1, Ua.shape[1]))]) - Ua
            out.append(np.stack([rom.sf.gamma[j] @ dU[j] for j in range(rom.k)]))
        return out

    def exchange(self, phis: List[np.ndarray], subset: Optional[Sequence[int]] = None) -> np.ndarray:
        """Step 2.1: sum the boundary-layer fluxes [phi_1]_f of every side of each port."""
        total = np.zeros(self.n_ports)
        for a in (range(len(self.subs)) if subset is None else subset):
            np.add.at(total, self.port_ids[a], phis[a][0])
        return total

    def accel(self, U: List[np.ndarray], fvals: Sequence[float] = ()) -> List[np.ndarray]:
        """Right-hand side a(U, t) of the coupled scheme (steps 2.1-2.3)."""
        phis = self.fluxes(U)
        port_flux = self.exchange(phis)
        return self._finish(U, phis, port_flux, fvals)

    def _finish(self, U, phis, port_flux, fvals):
        port_src = np.zeros(self.n_ports)
        for (a, vec, w), fv in zip(self.sources, fvals):
            port_src += fv * w
        acc = []
        for a, (rom, phi) in enumerate(zip(self.roms, phis)):
            out = np.zeros_like(U[a])
            for j in range(1, rom.k):                       # step 2.2, interior layers
                out[j] = rom.sf.gamma_hat[j] @ (phi[j] - phi[j - 1])
            ids = self.port_ids[a]                          # step 2.3, boundary layer
            out[0] = self.C[ids] * (port_flux[ids] + port_src[ids])
            acc.append(out)
        for (a, vec, w), fv in zip(self.sources, fvals):
            acc[a][1:] += fv * vec[1:]
        return acc

    def zero_state(self) -> List[np.ndarray]:
        return [np.zeros((rom.k, rom.p)) for rom in self.roms]

    def record(self, U: List[np.ndarray]) -> np.ndarray:
        return np.array([np.sum(row * U[a]) for a, row in self.receivers])

    def run(self, dt: float, wavelets: np.ndarray, U0: Optional[List[np.ndarray]] = None,
            U_prev: Optional[List[np.ndarray]] = None, return_state: bool = False):
        """Leapfrog; traces [nrec][nsteps], sample n recorded after the update to t_{n+1}."""
        wavelets = np.asarray(wavelets, dtype=np.float64).reshape(len(wavelets), -1)
        nsteps = wavelets.shape[0]
        U = [u.copy() for u in U0] if U0 is not None else self.zero_state()
        Up = [u.copy() for u in U_prev] if U_prev is not None else [u.copy() for u in U]
        traces = np.empty((len(self.receivers), nsteps))
        for n in range(nsteps):
            fv = wavelets[n] if self.sources else ()
            acc = self.accel(U, fv)
            Un = [2.0 * u - up + dt * dt * a for u, up, a in zip(U, Up, acc)]
            Up, U = U, Un
            traces[:, n] = self.record(U)
        if return_state:
            return traces, U, Up
        return traces

    # ------------------------------------------------------------------ assembled form
    def _dof_layout(self):
        offs = []
        o = self.n_ports
        for rom in self.roms:
            offs.append(o)
            o += (rom.k - 1) * rom.p
        return offs, o

    def gather(self, U: List[np.ndarray]) -> np.ndarray:
        """Global vector X = [ports; interior layers of every subdomain] from per-subdomain U."""
        offs, n = self._dof_layout()
        X = np.zeros(n)
        for a, Ua in enumerate(U):
            X[self.port_ids[a]] = Ua[0]
            X[offs[a]:offs[a] + Ua[1:].size] = Ua[1:].ravel()
        return X

    def scatter(self, X: np.ndarray) -> List[np.ndarray]:
        offs, _ = self._dof_layout()
        out = []
        for a, rom in enumerate(self.roms):
            Ua = np.empty((rom.k, rom.p))
            Ua[0] = X[self.port_ids[a]]
            Ua[1:] = X[offs[a]:offs[a] + (rom.k - 1) * rom.p].reshape(rom.k - 1, rom.p)
            out.append(Ua)
        return out

    def assemble(self):
        """Global (M, K, b): M X_tt = -K X + sum_s f_s b_s, summed over subdomains.

        Each subdomain contributes P^T Gamma-hat^{-1} P to M and P^T D^T Gamma D P to K,
        where P gathers its layer vectors from X (boundary layer from the ports).
        """
        from .sfraction import difference_stiffness
        offs, n = self._dof_layout()
        Mrows, Mcols, Mvals = [], [], []
        Krows, Kcols, Kvals = [], [], []
        for a, rom in enumerate(self.roms):
            k, p = rom.k, rom.p
            gidx = np.concatenate([self.port_ids[a], offs[a] + np.arange((k - 1) * p)])
            Minv_blocks = [np.diag(1.0 / self.H[a])] + [np.linalg.inv(rom.sf.gamma_hat[j])
                                                        for j in range(1, k)]
            for j, blk in enumerate(Minv_blocks):
                ii = gidx[j * p:(j + 1) * p]
                Mrows.append(np.repeat(ii, p)); Mcols.append(np.tile(ii, p)); Mvals.append(blk.ravel())
            Kloc = difference_stiffness(rom.sf)
            Krows.append(np.repeat(gidx, k * p)); Kcols.append(np.tile(gidx, k * p))
            Kvals.append(Kloc.ravel())
        M = sp.coo_matrix((np.concatenate(Mvals), (np.concatenate(Mrows), np.concatenate(Mcols))),
                          shape=(n, n)).tocsr()
        K = sp.coo_matrix((np.concatenate(Kvals), (np.concatenate(Krows), np.concatenate(Kcols))),
                          shape=(n, n)).tocsr()
        bs = []
        for a, vec, w in self.sources:
            rom = self.roms[a]
            Ua = [np.zeros((r.k, r.p)) for r in self.roms]
            # Gamma-hat^{-1} s on the source subdomain, summed into the global vector.
            b = np.zeros(n)
            b[self.port_ids[a]] += vec[0] / self.H[a]
            b[offs[a]:offs[a] + (rom.k - 1) * rom.p] = np.concatenate(
                [np.linalg.solve(rom.sf.gamma_hat[j], vec[j]) for j in range(1, rom.k)])
            bs.append(b)
        return M, K, bs

    def inverse_mass_factor(self) -> sp.csr_matrix:
        """L with L L^T = M^{-1}: sqrt(C) on the ports and chol(Gamma-hat_j) on interior blocks.

        M^{-1} is available blockwise without inverting Gamma-hat_j, which can be
        ill-conditioned for large j."""
        offs, n = self._dof_layout()
        rows, cols, vals = [np.arange(self.n_ports)], [np.arange(self.n_ports)], [np.sqrt(self.C)]
        for a, rom in enumerate(self.roms):
            p = rom.p
            for j in range(1, rom.k):
                Lj = np.linalg.cholesky(rom.sf.gamma_hat[j])
                ii = offs[a] + (j - 1) * p + np.arange(p)
                rows.append(np.repeat(ii, p)); cols.append(np.tile(ii, p)); vals.append(Lj.ravel())
        return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n)).tocsr()

    def max_eig(self) -> float:
        """rho = largest eigenvalue of M^{-1} K, computed as that of L^T K L (L L^T = M^{-1})."""
        _, K, _ = self.assemble()
        L = self.inverse_mass_factor()
        S = (L.T @ K @ L)
        n = S.shape[0]
        if n <= 6000:
            Sd = S.toarray()
            return float(sla.eigh(0.5 * (Sd + Sd.T), eigvals_only=True, subset_by_index=[n - 1, n - 1])[0])
        from scipy.sparse.linalg import eigsh
        return float(eigsh(S, k=1, which="LA", return_eigenvectors=False)[0])

    def cfl_dt(self) -> float:
        """Leapfrog stability limit dt_max = 2 / sqrt(rho)."""
        return 2.0 / np.sqrt(self.max_eig())

    def energy(self, M, K, X_new: np.ndarray, X_old: np.ndarray, dt: float) -> float:
        """Conserved leapfrog energy at t_{n+1/2}: 1/2 |X^{n+1}-X^n|_M^2 / dt^2 + 1/2 X^{n+1,T} K X^n."""
        d = X_new - X_old
        return 0.5 * d @ (M @ d) / (dt * dt) + 0.5 * X_new @ (K @ X_old)


def subdomain_bound(roms: List[SubdomainROM]) -> float:
    """max over subdomains of lambda_max(T^alpha); bounds rho of the coupled system (mediant of
    Rayleigh quotients of the per-subdomain terms)."""
    out = 0.0
    for rom in roms:
        out = max(out, float(np.linalg.eigvalsh(rom.tri.T())[-1]))
    return out

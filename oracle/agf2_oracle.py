"""Plain FP64 CPU oracle for AGF2(1,0) (Backhouse, Santana-Bonilla & Booth,
"Scalable and predictive spectra of correlated molecules with moment truncated
iterated perturbation theory", arXiv 2106.03508).

TEST INFRASTRUCTURE ONLY. Nothing in the product library may import, call or
link this file; only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the GPU path: numpy and LAPACK
(through numpy.linalg) only, float64 throughout, no blocking or fusion beyond
what each definition states.

Notation follows the paper: N physical orbitals (p, q, x, y), a Green's
function written as poles (energies lam, physical amplitudes u[N, npole]),
occupied poles i, j (below the chemical potential) and virtual poles a, b.
The DF tensor L[Q, p, q] factorises (pq|rs) = sum_Q L[Q,p,q] L[Q,r,s].

Readings of passages the paper leaves open are marked "Reading:" where used.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# Integrals and the Fock matrix
# ----------------------------------------------------------------------------

def eri_4index(L):
    """(pq|rs) = sum_Q L[Q,p,q] L[Q,r,s] as a dense [N,N,N,N] array
    (density fitting, the factorisation the cost analysis assumes)."""
    return np.einsum("Qpq,Qrs->pqrs", L, L, optimize=True)


def coulomb_exchange(L, D):
    """J_pq = sum_rs (pq|rs) D_rs and K_pq = sum_rs (ps|rq) D_rs, DF form."""
    rho = np.einsum("Qrs,rs->Q", L, D)
    J = np.einsum("Q,Qpq->pq", rho, L)
    K = np.einsum("Qps,sr,Qrq->pq", L, D, L, optimize=True)
    return J, K


def fock_matrix(h, L, D):
    """Generalised Fock matrix of the paper's Fock-matrix equation (section
    reviewing the method): F = h + sum_rs [(pq|rs) - 1/2 (ps|rq)] D_rs, with D
    the spin-summed one-body density matrix."""
    J, K = coulomb_exchange(L, D)
    return h + J - 0.5 * K


def synthetic_hcore(eps, L, nocc):
    """Reading: a synthetic system has no one-electron Hamiltonian of its own.
    Choose h so that the closed-shell determinant D0 = 2 * diag(1_occ) is a
    self-consistent mean-field solution with orbital energies eps:
    F[D0] = diag(eps) exactly (Fock-matrix equation solved for h)."""
    N = eps.shape[0]
    D0 = np.zeros((N, N))
    D0[np.arange(nocc), np.arange(nocc)] = 2.0
    J, K = coulomb_exchange(L, D0)
    return np.diag(eps) - J + 0.5 * K


def reference_density(nmo, nocc):
    D0 = np.zeros((nmo, nmo))
    D0[np.arange(nocc), np.arange(nocc)] = 2.0
    return D0


# ----------------------------------------------------------------------------
# Self-energy moments (zeroth- and first-moment equations; second-order
# self-energy equation for the lesser/greater split)
# ----------------------------------------------------------------------------

def pole_basis_df(L, u_pole, nocc_pole):
    """DF tensors in the pole basis: Lxo[Q,x,i] = sum_r L[Q,x,r] u[r,i],
    Lxv[Q,x,a] likewise, Lov[Q,i,a] = sum_xr u[x,i] L[Q,x,r] u[r,a]."""
    Q, N, _ = L.shape
    uo = np.ascontiguousarray(u_pole[:, :nocc_pole])
    uv = np.ascontiguousarray(u_pole[:, nocc_pole:])
    Lm = L.reshape(Q * N, N)
    Lxo = (Lm @ uo).reshape(Q, N, -1)
    Lxv = (Lm @ uv).reshape(Q, N, -1)
    Lov = np.empty((Q, uo.shape[1], uv.shape[1]))
    for q in range(Q):
        Lov[q] = uo.T @ Lxv[q]
    return Lxo, Lxv, Lov


def se_moments(L, e_pole, u_pole, nocc_pole, occ_sel=None, vir_sel=None, tensors=None):
    """Zeroth and first moments of the lesser and greater second-order
    self-energy, built from the Green's function poles (e_pole, u_pole).

    Lesser (first term of the second-order self-energy equation; the
    zeroth/first moment equations):
        U0<_pq = sum_{ija} (pi|ja) [2 (qi|ja) - (qj|ia)]
        U1<_pq = same summand times (e_i + e_j - e_a)
    Greater (second term; "analogous expressions" after the Cholesky step):
        U0>_pq = sum_{abi} (pa|bi) [2 (qa|bi) - (qb|ai)]
        U1>_pq = same summand times (e_a + e_b - e_i)
    Reading: at self-consistent iterations i, j, a, b run over the occupied
    and virtual poles of the dressed Green's function, with the integrals
    transformed by the poles' physical amplitudes u and weighted by the pole
    energies.

    Evaluated literally, one summed pole at a time, with the integrals taken
    from the DF factorisation. occ_sel / vir_sel restrict the outermost sum
    (over i for the lesser part, over a for the greater part) to a subset of
    poles; the full moments are the sums of these partial contributions.
    tensors, if given, is the output of pole_basis_df for these poles (reused
    instead of transforming again).
    Returns (U0<, U1<, U0>, U1>).
    """
    N = u_pole.shape[0]
    Q = L.shape[0]
    eo = e_pole[:nocc_pole]
    ev = e_pole[nocc_pole:]
    o, v = eo.shape[0], ev.shape[0]
    Lxo, Lxv, Lov = pole_basis_df(L, u_pole, nocc_pole) if tensors is None else tensors
    Lxo_m = np.ascontiguousarray(Lxo.reshape(Q, N * o))       # [Q, (x,j)]
    Lxv_m = np.ascontiguousarray(Lxv.reshape(Q, N * v))       # [Q, (x,b)]
    Lov_m = np.ascontiguousarray(Lov.reshape(Q, o * v))       # [Q, (j,a)]
    Lvo_m = np.ascontiguousarray(Lov.transpose(0, 2, 1).reshape(Q, v * o))  # [Q, (b,i)]
    m0o = np.zeros((N, N)); m1o = np.zeros((N, N))
    m0v = np.zeros((N, N)); m1v = np.zeros((N, N))
    for i in (range(o) if occ_sel is None else occ_sel):
        xija = (np.ascontiguousarray(Lxo[:, :, i].T) @ Lov_m).reshape(N, o, v)   # (xi|ja)
        xjia = (Lxo_m.T @ np.ascontiguousarray(Lov[:, i, :])).reshape(N, o, v)   # (xj|ia)
        w = eo[i] + eo[:, None] - ev[None, :]
        a = xija.reshape(N, -1)
        t = (2.0 * xija - xjia).reshape(N, -1)
        m0o += a @ t.T
        m1o += (a * w.reshape(1, -1)) @ t.T
    for a_ in (range(v) if vir_sel is None else vir_sel):
        xabi = (np.ascontiguousarray(Lxv[:, :, a_].T) @ Lvo_m).reshape(N, v, o)  # (xa|bi)
        xbai = (Lxv_m.T @ np.ascontiguousarray(Lov[:, :, a_])).reshape(N, v, o)  # (xb|ai)
        w = ev[a_] + ev[:, None] - eo[None, :]
        a = xabi.reshape(N, -1)
        t = (2.0 * xabi - xbai).reshape(N, -1)
        m0v += a @ t.T
        m1v += (a * w.reshape(1, -1)) @ t.T
    return m0o, m1o, m0v, m1v


def se_moments_n(L, e_pole, u_pole, nocc_pole, nmom):
    """Spectral moments 0..nmom-1 of the lesser and greater second-order
    self-energy (the moment equations of the compression section, continued
    to higher orders: the n-th moment carries the n-th power of the same
    weight),
        U<(n)_pq = sum_{ija} (pi|ja) [2 (qi|ja) - (qj|ia)] (e_i + e_j - e_a)^n
        U>(n)_pq = sum_{abi} (pa|bi) [2 (qa|bi) - (qb|ai)] (e_a + e_b - e_i)^n
    evaluated literally, one outer summed pole at a time, exactly as
    se_moments (which is nmom = 2). Moments 0 .. 2k+1 are what a compression
    to k + 1 Lanczos blocks conserves (the truncation family the paper names
    AGF2(n,m), n the number of conserved self-energy moment blocks).
    Returns (U< [nmom, N, N], U> [nmom, N, N])."""
    N = u_pole.shape[0]
    Q = L.shape[0]
    eo = e_pole[:nocc_pole]
    ev = e_pole[nocc_pole:]
    o, v = eo.shape[0], ev.shape[0]
    Lxo, Lxv, Lov = pole_basis_df(L, u_pole, nocc_pole)
    Lxo_m = np.ascontiguousarray(Lxo.reshape(Q, N * o))
    Lxv_m = np.ascontiguousarray(Lxv.reshape(Q, N * v))
    Lov_m = np.ascontiguousarray(Lov.reshape(Q, o * v))
    Lvo_m = np.ascontiguousarray(Lov.transpose(0, 2, 1).reshape(Q, v * o))
    mo = np.zeros((nmom, N, N))
    mv = np.zeros((nmom, N, N))
    for i in range(o):
        xija = (np.ascontiguousarray(Lxo[:, :, i].T) @ Lov_m).reshape(N, o, v)
        xjia = (Lxo_m.T @ np.ascontiguousarray(Lov[:, i, :])).reshape(N, o, v)
        w = (eo[i] + eo[:, None] - ev[None, :]).reshape(1, -1)
        a = xija.reshape(N, -1)
        t = (2.0 * xija - xjia).reshape(N, -1)
        for n in range(nmom):
            mo[n] += (a * w ** n) @ t.T
    for a_ in range(v):
        xabi = (np.ascontiguousarray(Lxv[:, :, a_].T) @ Lvo_m).reshape(N, v, o)
        xbai = (Lxv_m.T @ np.ascontiguousarray(Lov[:, :, a_])).reshape(N, v, o)
        w = (ev[a_] + ev[:, None] - eo[None, :]).reshape(1, -1)
        a = xabi.reshape(N, -1)
        t = (2.0 * xabi - xbai).reshape(N, -1)
        for n in range(nmom):
            mv[n] += (a * w ** n) @ t.T
    return mo, mv


def se_moment_elements(L, e_pole, u_pole, nocc_pole, pairs, progress=None):
    """Selected elements (p, q) of the four moments, each evaluated from the
    same literal sums as se_moments but only for the physical rows p and q
    involved (for sampling moments of systems too large to build whole).
    progress, if given, is called with a short text now and then.
    Returns an array [len(pairs), 4] of (U0<, U1<, U0>, U1>) values."""
    Q = L.shape[0]
    eo = e_pole[:nocc_pole]
    ev = e_pole[nocc_pole:]
    o, v = eo.shape[0], ev.shape[0]
    uo = u_pole[:, :nocc_pole]
    uv = u_pole[:, nocc_pole:]
    rows = sorted({p for p, _ in pairs} | {q for _, q in pairs})
    Lr = L[:, rows, :]                                          # [Q, rows, N]
    Lxo_r = np.einsum("Qxr,ri->Qxi", Lr, uo, optimize=True)     # (xi|Q) for the rows
    Lxv_r = np.einsum("Qxr,ra->Qxa", Lr, uv, optimize=True)
    # (ia|Q) = u_i^T L_Q u_a, one Q at a time
    Lov = np.empty((Q, o, v))
    for q in range(Q):
        Lov[q] = uo.T @ (L[q] @ uv)
        if progress and q % 500 == 499:
            progress(f"oracle transform {q + 1}/{Q}")
    Lov_m = Lov.reshape(Q, o * v)
    Lvo_m = np.ascontiguousarray(Lov.transpose(0, 2, 1).reshape(Q, v * o))
    Lov_i = np.ascontiguousarray(Lov.transpose(1, 0, 2))       # [o][Q][v]
    Lov_a = np.ascontiguousarray(Lov.transpose(2, 0, 1))       # [v][Q][o]
    pos = {x: k for k, x in enumerate(rows)}
    out = np.zeros((len(pairs), 4))
    w_o = eo[:, None, None] + eo[None, :, None] - ev[None, None, :]   # [i, j, a]
    w_v = ev[:, None, None] + ev[None, :, None] - eo[None, None, :]   # [a, b, i]
    for k, (p, q) in enumerate(pairs):
        rp, rq = pos[p], pos[q]
        # lesser: X[i, j, a] = (pi|ja), Y[i, j, a] = (qi|ja), E[i, j, a] = (qj|ia)
        X = (np.ascontiguousarray(Lxo_r[:, rp, :].T) @ Lov_m).reshape(o, o, v)
        Y = (np.ascontiguousarray(Lxo_r[:, rq, :].T) @ Lov_m).reshape(o, o, v)
        E = np.matmul(np.ascontiguousarray(Lxo_r[:, rq, :].T), Lov_i)  # [i][j][a]
        t = 2.0 * Y - E
        out[k, 0] = np.sum(X * t)
        out[k, 1] = np.sum(X * w_o * t)
        # greater: X[a, b, i] = (pa|bi), Y[a, b, i] = (qa|bi), E[a, b, i] = (qb|ai)
        X = (np.ascontiguousarray(Lxv_r[:, rp, :].T) @ Lvo_m).reshape(v, v, o)
        Y = (np.ascontiguousarray(Lxv_r[:, rq, :].T) @ Lvo_m).reshape(v, v, o)
        E = np.matmul(np.ascontiguousarray(Lxv_r[:, rq, :].T), Lov_a)  # [a][b][i]
        t = 2.0 * Y - E
        out[k, 2] = np.sum(X * t)
        out[k, 3] = np.sum(X * w_v * t)
        if progress:
            progress(f"oracle element {k + 1}/{len(pairs)}")
    return out


def se_moments_4index(eri, e_pole, u_pole, nocc_pole):
    """The same moments from explicit four-index integrals, transformed to
    the pole basis and summed with plain loops over the summed poles.
    Independent of the DF slab route; for tiny systems only."""
    uo = u_pole[:, :nocc_pole]
    uv = u_pole[:, nocc_pole:]
    eo = e_pole[:nocc_pole]
    ev = e_pole[nocc_pole:]
    # (p i | j a) and (p a | b i), p physical
    ovo = np.einsum("pqrs,qi,rj,sa->pija", eri, uo, uo, uv, optimize=True)
    vvo = np.einsum("pqrs,qa,rb,si->pabi", eri, uv, uv, uo, optimize=True)
    N = eri.shape[0]
    o, v = eo.shape[0], ev.shape[0]
    m0o = np.zeros((N, N)); m1o = np.zeros((N, N))
    m0v = np.zeros((N, N)); m1v = np.zeros((N, N))
    for i in range(o):
        for j in range(o):
            for a in range(v):
                left = ovo[:, i, j, a]
                right = 2.0 * ovo[:, i, j, a] - ovo[:, j, i, a]
                outer = np.outer(left, right)
                m0o += outer
                m1o += outer * (eo[i] + eo[j] - ev[a])
    for a in range(v):
        for b in range(v):
            for i in range(o):
                left = vvo[:, a, b, i]
                right = 2.0 * vvo[:, a, b, i] - vvo[:, b, a, i]
                outer = np.outer(left, right)
                m0v += outer
                m1v += outer * (ev[a] + ev[b] - eo[i])
    return m0o, m1o, m0v, m1v


def uncompressed_self_energy(L, e_pole, u_pole, nocc_pole):
    """Explicit auxiliary (pole) form of the second-order self-energy,
    Sigma_pq(w) = sum_k v_pk v_qk / (w - E_k) (auxiliary self-energy
    equation), for tiny systems. The exchange-weighted numerator
    X^{ij} (2X^{ij} - X^{ji})^T, summed over an (i, j) pair and its mirror,
    is a sum of squares: with P = X^{ij} + X^{ji}, M = X^{ij} - X^{ji} it is
    1/2 P P^T + 3/2 M M^T, and X^{ii} X^{ii T} on the diagonal, where
    X^{ij}[x, a] = (xi|ja). Each column is one auxiliary with energy
    e_i + e_j - e_a (lesser) or e_a + e_b - e_i (greater).

    Returns (E<, v<, E>, v>) with v of shape [N, naux]."""
    Lxo, Lxv, Lov = pole_basis_df(L, u_pole, nocc_pole)
    eo = e_pole[:nocc_pole]
    ev = e_pole[nocc_pole:]

    def build(Lx, Lpc, ep, ec, sign):
        # X[p][q][x, c] = sum_Q Lx[Q,x,p] Lpc(q)[Q,c]
        n = ep.shape[0]
        E, V = [], []
        for p in range(n):
            for q in range(p, n):
                Xpq = Lx[:, :, p].T @ Lpc(q)   # [x, c]
                if p == q:
                    for c in range(ec.shape[0]):
                        V.append(Xpq[:, c]); E.append(ep[p] + ep[p] - ec[c])
                    continue
                Xqp = Lx[:, :, q].T @ Lpc(p)
                for c in range(ec.shape[0]):
                    V.append(np.sqrt(0.5) * (Xpq[:, c] + Xqp[:, c]))
                    E.append(ep[p] + ep[q] - ec[c])
                    V.append(np.sqrt(1.5) * (Xpq[:, c] - Xqp[:, c]))
                    E.append(ep[p] + ep[q] - ec[c])
        return np.array(E), np.array(V).T

    Eo, Vo = build(Lxo, lambda j: Lov[:, j, :], eo, ev, +1)
    Ev, Vv = build(Lxv, lambda b: Lov[:, :, b], ev, eo, -1)
    return Eo, Vo, Ev, Vv


def mp2_energy_bruteforce(eri, eps, nocc):
    """Closed-shell MP2 correlation energy with plain loops:
    sum_{ijab} (ia|jb)[2(ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)."""
    N = eps.shape[0]
    e = 0.0
    for i in range(nocc):
        for j in range(nocc):
            for a in range(nocc, N):
                for b in range(nocc, N):
                    iajb = eri[i, a, j, b]
                    ibja = eri[i, b, j, a]
                    e += iajb * (2.0 * iajb - ibja) / (eps[i] + eps[j] - eps[a] - eps[b])
    return e


# ----------------------------------------------------------------------------
# Compression: one block-Lanczos step through a Cholesky factor
# ----------------------------------------------------------------------------

class NotPositiveDefinite(RuntimeError):
    pass


def compress(m0, m1, tol=0.0):
    """Auxiliaries conserving the zeroth and first moments (block Lanczos,
    single step, via Cholesky; compression section).

    Reading: the paper writes T T^dagger = U0 and M = (T^-1)^dagger U1 T^-1,
    which agree only for the upper factor. Any square root S with
    S S^T = U0 gives the same self-energy; take the lower Cholesky factor,
    M = S^-1 U1 S^-T, diagonalise M = W diag(e) W^T and couple the
    auxiliaries through v = S W, so v v^T = U0 and v diag(e) v^T = U1.

    tol == 0: strict Cholesky, NotPositiveDefinite on failure.
    tol > 0: square root from the eigendecomposition of U0 keeping
    eigenvalues above tol * max eigenvalue (fewer auxiliaries when U0 is
    singular).
    Returns (e[naux], v[N, naux])."""
    if tol == 0.0:
        try:
            S = np.linalg.cholesky(m0)
        except np.linalg.LinAlgError as exc:
            raise NotPositiveDefinite(str(exc)) from exc
        Sinv = np.linalg.inv(S)
        M = Sinv @ m1 @ Sinv.T
    else:
        s, Z = np.linalg.eigh(m0)
        keep = s > tol * s.max()
        if not np.any(keep):
            raise NotPositiveDefinite("zeroth moment has no positive eigenvalue")
        S = Z[:, keep] * np.sqrt(s[keep])
        Spinv = (Z[:, keep] / np.sqrt(s[keep])).T
        M = Spinv @ m1 @ Spinv.T
    M = 0.5 * (M + M.T)
    e, W = np.linalg.eigh(M)
    return e, S @ W


def block_lanczos(moments):
    """Compression of one part of the self-energy to nblock = len(moments)/2
    blocks of N auxiliaries that conserve its moments 0 .. 2 nblock - 1
    (the block-Lanczos compression of the compression section, run for
    more than one block: the other truncations of the AGF2(n,m) family).

    Reading: the self-energy part is Sigma(w) = V (w - E)^-1 V^T over its
    (uncompressed) auxiliaries, with moments T(n) = V E^n V^T. With
    S S^T = T(0) (lower Cholesky factor) the block Q0 = V^T S^-T is
    orthonormal and the moments of H = diag(E) seen from it are
    M(n) = Q0^T H^n Q0 = S^-1 T(n) S^-T (M(0) = I). Block Lanczos on H from
    Q0,
        H Q_j = Q_{j-1} B_j^T + Q_j A_j + Q_{j+1} B_{j+1},
    needs only these moments: each Q_j is a polynomial in H applied to Q0,
    Q_j = sum_m H^m Q0 C_j[m], so every inner product is
    <Q_i|H^p|Q_j> = sum_{m,l} C_i[m]^T M(m+l+p) C_j[l]. Here
    A_j = <Q_j|H|Q_j>; the residual R_{j+1} = H Q_j - Q_j A_j - Q_{j-1} B_j^T
    has coefficients shifted and combined from those of Q_j and Q_{j-1};
    B_{j+1} is the upper Cholesky factor of <R|R> (B^T B = <R|R>) and
    Q_{j+1} = R B^-1. A_k needs moments up to 2k+1 and B_k up to 2k.
    The block tridiagonal T (A_j on the diagonal, B_j below, B_j^T above)
    is diagonalised, T = W diag(e) W^T; the compressed auxiliaries are
    e and v = S W[:N], so that v diag(e)^n v^T = S (T^n)_00 S^T = T(n) for
    n <= 2 nblock - 1. One block is compress(T(0), T(1)).
    Raises NotPositiveDefinite when T(0) or a <R|R> is not positive
    definite. Returns (e [nblock N], v [N, nblock N])."""
    nm = len(moments)
    if nm < 2 or nm % 2:
        raise ValueError("need an even number of moments")
    nblock = nm // 2
    N = moments[0].shape[0]
    try:
        S = np.linalg.cholesky(moments[0])
    except np.linalg.LinAlgError as exc:
        raise NotPositiveDefinite(str(exc)) from exc
    Sinv = np.linalg.inv(S)
    M = [Sinv @ T @ Sinv.T for T in moments]
    M = [0.5 * (x + x.T) for x in M]

    def inner(Ci, Cj, p):
        out = np.zeros((N, N))
        for m, cm in enumerate(Ci):
            for l, cl in enumerate(Cj):
                out += cm.T @ M[m + l + p] @ cl
        return out

    C = [[np.eye(N)]]
    A = [inner(C[0], C[0], 1)]
    B = []
    for j in range(1, nblock):
        R = [np.zeros((N, N)) for _ in range(j + 1)]
        for m, cm in enumerate(C[j - 1]):
            R[m + 1] += cm                       # H Q_{j-1}
            R[m] -= cm @ A[j - 1]                # - Q_{j-1} A_{j-1}
        if j >= 2:
            for m, cm in enumerate(C[j - 2]):
                R[m] -= cm @ B[j - 2].T          # - Q_{j-2} B_{j-1}^T
        G = inner(R, R, 0)
        try:
            Lc = np.linalg.cholesky(0.5 * (G + G.T))
        except np.linalg.LinAlgError as exc:
            raise NotPositiveDefinite(f"block {j}: {exc}") from exc
        Bj = Lc.T
        Binv = np.linalg.inv(Bj)
        C.append([r @ Binv for r in R])
        B.append(Bj)
        A.append(inner(C[j], C[j], 1))
    T = np.zeros((nblock * N, nblock * N))
    for j in range(nblock):
        T[j * N:(j + 1) * N, j * N:(j + 1) * N] = 0.5 * (A[j] + A[j].T)
    for j in range(1, nblock):
        T[j * N:(j + 1) * N, (j - 1) * N:j * N] = B[j - 1]
        T[(j - 1) * N:j * N, j * N:(j + 1) * N] = B[j - 1].T
    e, W = np.linalg.eigh(T)
    return e, S @ W[:N]


def self_energy_at(w, e_aux, v_aux):
    """Sigma(w) = sum_k v_k v_k^T / (w - e_k) (auxiliary self-energy eq.)."""
    return (v_aux / (w - e_aux)) @ v_aux.T


# ----------------------------------------------------------------------------
# Fock loop: extended Fock matrix, aufbau, chemical potential, density
# ----------------------------------------------------------------------------

def extended_hamiltonian(F, e_aux, v_aux):
    """[[F, v], [v^T, diag(e)]] (compressed extended Hamiltonian equation)."""
    N = F.shape[0]
    n = e_aux.shape[0]
    H = np.zeros((N + n, N + n))
    H[:N, :N] = F
    H[:N, N:] = v_aux
    H[N:, :N] = v_aux.T
    H[N:, N:] = np.diag(e_aux)
    return H


def aufbau(lam, u, nelec):
    """Reading: fill the poles in ascending energy, two electrons times each
    pole's physical weight |u_l|^2; the occupied count n* minimises
    |c_n - nelec| with c_n = 2 sum_{l<n} |u_l|^2 (ties -> smaller n). The
    chemical potential sits midway between the last occupied and first
    virtual pole. Returns (n*, c_{n*}, mu)."""
    w = np.sum(u * u, axis=0)
    c = 2.0 * np.concatenate([[0.0], np.cumsum(w)])
    n = int(np.argmin(np.abs(c - nelec)))
    npole = lam.shape[0]
    if 0 < n < npole:
        mu = 0.5 * (lam[n - 1] + lam[n])
    elif n == 0:
        mu = lam[0] - 1.0
    else:
        mu = lam[-1] + 1.0
    return n, c[n], mu


def _solve(F, e_aux, v_aux, shift, nelec):
    H = extended_hamiltonian(F, e_aux + shift, v_aux)
    lam, phi = np.linalg.eigh(H)
    N = F.shape[0]
    u = phi[:N]
    n, cnt, mu = aufbau(lam, u, nelec)
    return lam, u, n, cnt, mu


def fit_shift(F, e_aux, v_aux, nelec, shift0=0.0, bracket=2.0, tol=1e-10,
              step0=0.01, max_iter=200):
    """Reading of the chemical-potential condition (electron number kept
    exact in a non-idempotent density): shift every auxiliary energy by a
    common Delta until the aufbau count equals nelec.

    For a fixed number n of occupied poles, c_n(Delta) is non-decreasing in
    Delta (the sum of the n lowest eigenvalues is concave in Delta and its
    derivative is n - c_n/2), so the root of g(Delta) = c_n(Delta) - nelec is
    bracketed by stepping away from shift0 (step0, doubling, never beyond
    shift0 +- bracket) and then found by bisection, stopping when |g| < tol.
    If the aufbau picks another n at the root, repeat with that n.
    Returns (shift, n_eig) with n_eig the number of eigensolves used."""
    n_eig = 1
    lam, u, n, cnt, mu = _solve(F, e_aux, v_aux, shift0, nelec)
    shift = shift0
    for _ in range(8):
        g0 = cnt - nelec
        if abs(g0) < tol:
            return shift, n_eig

        def g(d):
            lam_, u_, nn_, cnt_, mu_ = _solve(F, e_aux, v_aux, d, nelec)
            return 2.0 * np.sum(u_[:, :n] ** 2) - nelec

        # bracket: g is non-decreasing, so move up when g < 0
        direction = 1.0 if g0 < 0 else -1.0
        a, ga = shift, g0
        step = step0
        while True:
            b = shift + direction * min(step, bracket)
            gb = g(b); n_eig += 1
            if gb == 0.0 or (gb > 0) != (ga > 0) or step >= bracket:
                break
            a, ga = b, gb
            step *= 2.0
        if (gb > 0) == (ga > 0) and gb != 0.0:
            x = b              # no sign change inside the allowed bracket
        else:
            # bisection on [a, b]; g(a) and g(b) have opposite signs
            x = b
            for _ in range(max_iter):
                if gb == 0.0 or abs(gb) < tol:
                    x = b
                    break
                x = 0.5 * (a + b)
                gx = g(x); n_eig += 1
                if abs(gx) < tol:
                    break
                if (gx > 0) == (ga > 0):
                    a, ga = x, gx
                else:
                    b, gb = x, gx
        shift = x
        lam, u, n_new, cnt, mu = _solve(F, e_aux, v_aux, shift, nelec)
        n_eig += 1
        if n_new == n:
            return shift, n_eig
        n = n_new
    return shift, n_eig


def fock_loop(h, L, nelec, e_aux, v_aux, D, tol_rdm1=1e-8, tol_nelec=1e-10,
              max_cycle=50, bracket=2.0, shift0=0.0, diis_space=8, step0=0.01):
    """Density relaxation with the chemical potential held at the right
    electron number (relaxation passage after the self-consistency
    discussion), on the compressed extended Hamiltonian.

    Each cycle: Delta fitted at the current F to |count - nelec| < tol_nelec
    (fit_shift); eigendecomposition of [[F, v], [v^T, diag(e + Delta)]];
    aufbau; D = 2 sum_{l<n*} u_l u_l^T; stop when the Frobenius norm of the
    change of D is below tol_rdm1, else the next F is F[D], DIIS-extrapolated
    with the fixed-point residual F[D] - F as error.
    Reading: the tolerance bounds the whole change of the density matrix, so
    the energy it leaves unconverged does not grow with the basis size.
    The returned F is the one diagonalised last, so the returned poles are
    exact eigenpairs of the returned extended Hamiltonian. When max_cycle is
    reached first, the shift is fitted once more at the last F and the poles
    and density returned are those of that F (converged False).
    Returns a dict."""
    F = fock_matrix(h, L, D)
    shift = shift0
    n_eig = 0
    converged = False
    diis = DIIS(diis_space) if diis_space else None
    N = F.shape[0]
    for cycle in range(1, max_cycle + 1):
        shift, ne = fit_shift(F, e_aux, v_aux, nelec, shift0=shift, bracket=bracket,
                              tol=tol_nelec, step0=step0)
        n_eig += ne
        lam, u, n, cnt, mu = _solve(F, e_aux, v_aux, shift, nelec)
        n_eig += 1
        uo = u[:, :n]
        D_new = 2.0 * uo @ uo.T
        err = np.linalg.norm(D_new - D)
        D = D_new
        if err < tol_rdm1:
            converged = True
            break
        F_new = fock_matrix(h, L, D)
        if diis is not None:
            F_new = diis.update(F_new, err=F_new - F).reshape(N, N)
        F = F_new
    if not converged:
        shift, ne = fit_shift(F, e_aux, v_aux, nelec, shift0=shift, bracket=bracket,
                              tol=tol_nelec, step0=step0)
        n_eig += ne
        lam, u, n, cnt, mu = _solve(F, e_aux, v_aux, shift, nelec)
        n_eig += 1
        uo = u[:, :n]
        D = 2.0 * uo @ uo.T
    return dict(e_pole=lam, u_pole=u, nocc_pole=n, mu=mu, shift=shift,
                rdm1=D, fock=F, n_cycle=cycle, n_eig=n_eig, converged=converged,
                nelec=cnt)


# ----------------------------------------------------------------------------
# Energy and observables
# ----------------------------------------------------------------------------

def energy_gf(h, F, D, e_pole, u_pole, nocc_pole, e_occ_aux, v_occ_aux,
              e_vir_aux, v_vir_aux):
    """Galitskii-Migdal energy of a Green's function and its self-energy.

    Reading (the paper mentions static energetics but prints no formula):
    for poles (lam_l, u_l) that are eigenpairs of [[F, v], [v^T, diag(e)]],
    GM gives E = 1/2 Tr[(h + F) D] + sum_{l occ} sum_k (u_l.v_k)^2/(lam_l - e_k).
    Because sum over all l of (u_l.v_k)^2/(lam_l - e_k) vanishes for every
    auxiliary k (the physical-auxiliary block of the eigenvector completeness
    relation), the lesser-auxiliary part of that sum equals a virtual-pole
    sum, so
      E_2b = sum_{l occ} sum_{k>} (u_l.v_k)^2/(lam_l - e_k)
           + sum_{l vir} sum_{k<} (u_l.v_k)^2/(e_k - lam_l),
    which has no near-zero denominators. Returns (E_1b, E_2b)."""
    e1b = 0.5 * np.sum((h + F) * D)
    uo = u_pole[:, :nocc_pole]
    uv = u_pole[:, nocc_pole:]
    lo = e_pole[:nocc_pole]
    lv = e_pole[nocc_pole:]
    c_ov = (uo.T @ v_vir_aux) ** 2                        # [l occ, k >]
    e2b = np.sum(c_ov / (lo[:, None] - e_vir_aux[None, :]))
    c_vo = (uv.T @ v_occ_aux) ** 2                        # [l vir, k <]
    e2b += np.sum(c_vo / (e_occ_aux[None, :] - lv[:, None]))
    return e1b, e2b


def energy_gf_onesided_all(h, F, D, e_pole, u_pole, nocc_pole, e_aux, v_aux):
    """GM two-body term in its direct form, occupied poles against every
    auxiliary: sum_{l occ} sum_k (u_l.v_k)^2/(lam_l - e_k)."""
    uo = u_pole[:, :nocc_pole]
    lo = e_pole[:nocc_pole]
    c = (uo.T @ v_aux) ** 2
    return np.sum(c / (lo[:, None] - e_aux[None, :]))


def ip_ea(e_pole, u_pole, nocc_pole):
    """IP = -(energy of the highest occupied pole), EA = energy of the
    lowest virtual pole, with their quasiparticle weights |u|^2."""
    w = np.sum(u_pole * u_pole, axis=0)
    return (-e_pole[nocc_pole - 1], e_pole[nocc_pole],
            w[nocc_pole - 1], w[nocc_pole])


def spectral_function(e_pole, u_pole, omega, eta, weight=None):
    """Broadened spectral function in the physical space (the simulated
    photoelectron spectra of the artemisinin section, with a broadening
    factor eta): A(w) = -1/pi Im Tr[P G(w + i eta)].

    G(z) is the physical block of the resolvent of the extended Hamiltonian
    whose eigenpairs the Dyson equation gives (`dyson_eq_eig`), so
    G(z) = sum_l u_l u_l^T / (z - lam_l) and
      A(w) = eta/pi sum_l w_l / ((w - lam_l)^2 + eta^2),
      w_l  = sum_p P_p u[p, l]^2.
    Reading: P = diag(weight) is a weight per physical orbital (a projection
    such as the paper's atomic one, which needs basis data a synthetic
    system lacks); weight None is the identity, the total spectrum."""
    e_pole = np.asarray(e_pole, dtype=np.float64)
    u_pole = np.asarray(u_pole, dtype=np.float64)
    omega = np.asarray(omega, dtype=np.float64)
    P = np.ones(u_pole.shape[0]) if weight is None else np.asarray(weight, np.float64)
    w = np.sum(P[:, None] * u_pole * u_pole, axis=0)
    d = omega[:, None] - e_pole[None, :]
    return eta / np.pi * np.sum(w[None, :] / (d * d + eta * eta), axis=1)


# ----------------------------------------------------------------------------
# Outer self-consistency
# ----------------------------------------------------------------------------

class DIIS:
    """Pulay (DIIS) extrapolation over the last `space` iterates. The error
    vector of an iterate is either given, or taken as the change since the
    previous iterate."""

    def __init__(self, space=8):
        self.space = space
        self.xs = []
        self.es = []
        self.prev = None

    def update(self, x, err=None):
        x = np.asarray(x, dtype=np.float64).ravel()
        if err is None:
            if self.prev is None:
                self.prev = x.copy()
                return x
            e = x - self.prev
            self.prev = x.copy()
        else:
            e = np.asarray(err, dtype=np.float64).ravel()
        self.xs.append(x.copy()); self.es.append(e.copy())
        if len(self.xs) > self.space:
            self.xs.pop(0); self.es.pop(0)
        n = len(self.xs)
        if n < 2:
            return x
        B = np.zeros((n + 1, n + 1))
        for a in range(n):
            for b in range(n):
                B[a, b] = self.es[a] @ self.es[b]
        B[n, :n] = B[:n, n] = -1.0
        rhs = np.zeros(n + 1); rhs[n] = -1.0
        try:
            c = np.linalg.solve(B, rhs)[:n]
        except np.linalg.LinAlgError:
            return x
        out = np.zeros_like(x)
        for ci, xi in zip(c, self.xs):
            out += ci * xi
        return out


def run_agf2(h, L, eps, nocc, max_iter=20, conv_tol=1e-8, conv_tol_ipea=1e-7,
             diis_space=8, fock_opts=None, compress_tol=0.0, verbose=False, nblock=1):
    """AGF2(1,0) to self-consistency (the method as reviewed in the paper):
    start from the mean-field poles; each iteration builds the four moments
    from the current poles, extrapolates them (DIIS), compresses the lesser
    and greater parts to N auxiliaries each, relaxes the density in the Fock
    loop, and evaluates the energy and IP/EA. Converged when the energy
    changes by less than conv_tol and IP/EA by less than conv_tol_ipea.
    Stops unconverged when a Fock loop reaches its cycle limit.
    nblock > 1: each part is compressed to nblock Lanczos blocks conserving
    moments 0 .. 2 nblock - 1 (block_lanczos), so the Green's function has
    N + 2 nblock N poles."""
    fock_opts = dict(fock_opts or {})
    N = eps.shape[0]
    nelec = 2 * nocc
    e_pole = eps.copy()
    u_pole = np.eye(N)
    nocc_pole = nocc
    D = reference_density(N, nocc)
    diis = DIIS(diis_space) if diis_space else None
    hist = []
    prev = None
    converged = False
    nmom = 2 * nblock
    for it in range(max_iter + 1):
        if nblock == 1:
            m = se_moments(L, e_pole, u_pole, nocc_pole)
        else:
            mo, mv = se_moments_n(L, e_pole, u_pole, nocc_pole, nmom)
            m = tuple(mo) + tuple(mv)
        if diis is not None:
            flat = diis.update(np.concatenate([x.ravel() for x in m]))
            m = tuple(flat[k * N * N:(k + 1) * N * N].reshape(N, N) for k in range(2 * nmom))
        m = tuple(0.5 * (x + x.T) for x in m)
        if nblock == 1:
            eo, vo = compress(m[0], m[1], tol=compress_tol)
            ev, vv = compress(m[2], m[3], tol=compress_tol)
        else:
            eo, vo = block_lanczos(m[:nmom])
            ev, vv = block_lanczos(m[nmom:])
        e_aux = np.concatenate([eo, ev])
        v_aux = np.hstack([vo, vv])
        fl = fock_loop(h, L, nelec, e_aux, v_aux, D, **fock_opts)
        e_pole, u_pole, nocc_pole, D = fl["e_pole"], fl["u_pole"], fl["nocc_pole"], fl["rdm1"]
        shift = fl["shift"]
        e1b, e2b = energy_gf(h, fl["fock"], D, e_pole, u_pole, nocc_pole,
                             eo + shift, vo, ev + shift, vv)
        ip, ea, wip, wea = ip_ea(e_pole, u_pole, nocc_pole)
        rec = dict(iter=it, e1b=e1b, e2b=e2b, etot=e1b + e2b, ip=ip, ea=ea,
                   wip=wip, wea=wea, nocc_pole=nocc_pole, npole=e_pole.shape[0],
                   mu=fl["mu"], shift=shift, fock_cycles=fl["n_cycle"],
                   fock_eig=fl["n_eig"], fock_converged=fl["converged"])
        hist.append(rec)
        if verbose:
            print(rec)
        if not fl["converged"]:
            break              # the density of this iteration is not relaxed
        if prev is not None:
            if (abs(rec["etot"] - prev["etot"]) < conv_tol
                    and max(abs(ip - prev["ip"]), abs(ea - prev["ea"])) < conv_tol_ipea):
                converged = True
                break
        prev = rec
    return dict(history=hist, converged=converged, e_pole=e_pole, u_pole=u_pole,
                nocc_pole=nocc_pole, rdm1=D, e_aux=e_aux, v_aux=v_aux)

"""Pins of the plain CPU oracle against facts that do not come from the oracle:
closed forms, invariants, library routines the oracle does not use, brute
force on tiny grids and numbers printed in the paper (tests/golden/).

Each test names the passage of the paper (arXiv 2508.02613) it follows.
"""
import os

import numpy as np
import pytest

import jfft_inputs as ji
import oracle

LAM, MU = oracle.lame_from_nu(0.3)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        key, rest = parts[0], parts[1:]
        nums = []
        for p in rest:
            try:
                nums.append(float(p))
            except ValueError:
                break
        vals[key] = nums
    return vals


# ----------------------------------------------------------- closed forms --
def mandel_iso(dim, lam, mu):
    ds = dim * (dim + 1) // 2
    Cm = np.zeros((ds, ds))
    Cm[:dim, :dim] = lam
    Cm[np.arange(dim), np.arange(dim)] += 2 * mu
    Cm[np.arange(dim, ds), np.arange(dim, ds)] = 2 * mu
    return Cm


def symbol_closed_form(shape, lam, mu, lengths=None):
    """Fourier symbol of K_ref for Q1 elements with full 2-point Gauss
    integration, built from the tensor-product 1D stencils: stiffness
    (1/h)(-1, 2, -1) -> a = (2 - 2 cos t)/h, mass (h/6)(1, 4, 1) ->
    b = h (2 + cos t)/3, first-derivative coupling -> +-i sin t.  Reduces in 1D
    to the stencil (-1, 2, -1) of the appendix (eigenvalues 2 - 2 cos)."""
    dim = len(shape)
    n_xyz = shape[::-1]
    lengths = lengths or (1.0,) * dim
    A, B, S = [], [], []
    for ax in range(dim):
        n = n_xyz[ax]
        h = lengths[ax] / n
        t = 2 * np.pi * np.arange(n) / n
        bshape = [1] * dim
        bshape[dim - 1 - ax] = n
        A.append(((2 - 2 * np.cos(t)) / h).reshape(bshape))
        B.append((h * (2 + np.cos(t)) / 3).reshape(bshape))
        S.append(np.sin(t).reshape(bshape))
    K = np.zeros((dim, dim) + tuple(shape))
    for i in range(dim):
        others = [j for j in range(dim) if j != i]
        diag = (lam + 2 * mu) * A[i]
        for j in others:
            diag = diag * B[j]
        for j in others:
            term = mu * B[i] * A[j]
            for m in others:
                if m != j:
                    term = term * B[m]
            diag = diag + term
        K[i, i] = diag
        for j in others:
            term = (lam + mu) * S[i] * S[j]
            for m in range(dim):
                if m not in (i, j):
                    term = term * B[m]
            K[i, j] = term
    return K


def invert_blocks(K):
    d = K.shape[0]
    shape = K.shape[2:]
    G = np.zeros_like(K)
    Km = np.moveaxis(K.reshape(d, d, -1), -1, 0)
    Gm = np.zeros_like(Km)
    Gm[1:] = np.linalg.inv(Km[1:])
    return np.moveaxis(Gm, 0, -1).reshape((d, d) + shape)


def dense_K(E, lam, mu):
    dim = E.ndim
    ndof = dim * E.size
    K = np.zeros((ndof, ndof))
    for j in range(ndof):
        e = np.zeros(ndof)
        e[j] = 1.0
        K[:, j] = oracle.stiffness(E, e.reshape((dim,) + E.shape), lam, mu).ravel()
    return K


def element_matrix_kron(dim, h, lam, mu):
    """Q1 element stiffness on a cube of side h from 1D element matrices:
    k1 = (1/h)[[1,-1],[-1,1]], m1 = (h/6)[[2,1],[1,2]],
    g1[a, b] = int phi_a' phi_b = 0.5*[[-1,-1],[1,1]].  Local node order
    corner c = c0 + 2 c1 (+ 4 c2), dof = c*d + comp."""
    k1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    m1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6
    g1 = 0.5 * np.array([[-1.0, -1.0], [1.0, 1.0]])

    def kron_axes(mats):
        # mats[a] acts on axis a; corner bits c_a; kron order: highest axis first
        out = np.ones((1, 1))
        for a in reversed(range(dim)):
            out = np.kron(out, mats[a])
        return out

    def T(k, l):
        # int d_k phi_I d_l phi_J over the element
        mats = []
        for a in range(dim):
            if k == a and l == a:
                mats.append(k1)
            elif k == a:
                mats.append(g1)
            elif l == a:
                mats.append(g1.T)
            else:
                mats.append(m1)
        return kron_axes(mats)

    nloc = 2 ** dim
    Ke = np.zeros((dim * nloc, dim * nloc))
    for i in range(dim):
        for j in range(dim):
            blk = np.zeros((nloc, nloc))
            for k in range(dim):
                for l in range(dim):
                    cikjl = lam * (i == k) * (j == l) + mu * ((i == j) * (k == l) + (i == l) * (k == j))
                    if cikjl:
                        blk += cikjl * T(k, l)
            Ke[i::dim, j::dim] = blk
    return Ke


# ------------------------------------------------------------------- P15 --
def test_p15_dft_matches_library_and_closed_form():
    """Naive DFT of eq. prec_lin_systemG_FFT vs numpy.fft (a routine the
    oracle does not use) and vs the closed form of a cosine."""
    rng = np.random.default_rng(0)
    for shape in [(6, 10), (4, 6, 8), (3, 5, 7)]:
        x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        X = oracle.dft(x, -1)
        assert np.abs(X - np.fft.fftn(x)).max() <= 1e-12 * np.abs(X).max()
        y = oracle.dft(X, +1) / x.size
        assert np.abs(y - x).max() <= 1e-13 * np.abs(x).max()
    n = 12
    j = np.arange(n)
    c = np.cos(2 * np.pi * 3 * j / n)[None, :] * np.ones((4, 1))
    C = oracle.dft(c, -1)
    ref = np.zeros((4, n), complex)
    ref[0, 3] = ref[0, n - 3] = 4 * n / 2
    assert np.abs(C - ref).max() <= 1e-12


# -------------------------------------------------------------------- P7 --
@pytest.mark.parametrize("shape,lengths", [((8, 6), None), ((6, 4, 8), None),
                                           ((4, 6, 10), (1.0, 2.0, 0.5)), ((12, 10), (2.0, 1.0))])
def test_p7_alg1_green_symbol_closed_form(shape, lengths):
    """Algorithm 1 output equals the inverse of the closed-form Q1 symbol at
    k != 0 and zero at k = 0 (Alg. 1 step 3)."""
    G = oracle.green(shape, LAM, MU, lengths=lengths)
    Kc = symbol_closed_form(shape, LAM, MU, lengths=lengths)
    Gc = invert_blocks(Kc)
    assert np.abs(G.imag).max() <= 1e-12 * np.abs(G.real).max()
    assert np.abs(G.real - Gc).max() <= 1e-12 * np.abs(Gc).max()
    zero = (slice(None), slice(None)) + (0,) * len(shape)
    assert np.all(G[zero] == 0)
    # blocks are real symmetric, positive definite off k = 0 (reading A9)
    Km = np.moveaxis(Kc.reshape(len(shape), len(shape), -1), -1, 0)[1:]
    assert np.allclose(Km, np.swapaxes(Km, 1, 2))
    assert np.linalg.eigvalsh(Km).min() > 0


def test_p7_stiffness_on_fourier_mode():
    """With uniform E, K maps cos(2 pi k.x) e_alpha to the symbol times the mode."""
    shape = (6, 8, 10)
    kvec = (1, 2, 3)  # (kz, ky, kx)
    nz, ny, nx = shape
    Kc = symbol_closed_form(shape, LAM, MU)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = 2 * np.pi * (kvec[0] * zz / nz + kvec[1] * yy / ny + kvec[2] * xx / nx)
    for alpha in range(3):
        u = np.zeros((3,) + shape)
        u[alpha] = np.cos(phase)
        Ku = oracle.stiffness(np.ones(shape), u, LAM, MU)
        for beta in range(3):
            s = Kc[beta, alpha][kvec]
            # real symmetric, even symbol: diagonal blocks give s cos, odd-odd
            # off-diagonal products give s cos as well (sin_i sin_j)
            expect = s * np.cos(phase)
            assert np.abs(Ku[beta] - expect).max() <= 1e-12 * max(1.0, np.abs(Ku).max())


def test_element_stiffness_kronecker_closed_form():
    """Material on a single element: K equals E_e times the element matrix
    built from the 1D stiffness/mass/coupling matrices (eq. disc_wf with exact
    2-point Gauss integration)."""
    for dim, shape in [(2, (4, 4)), (3, (4, 4, 4))]:
        E = np.zeros(shape)
        idx = (1,) * dim
        E[idx] = 3.7
        K = dense_K(E, LAM, MU)
        n = shape[0]
        Ke = element_matrix_kron(dim, 1.0 / n, LAM, MU)
        nloc = 2 ** dim
        nodes = []
        for c in range(nloc):
            pos = [(1 + ((c >> a) & 1)) for a in range(dim)]  # x, y, z
            flat = 0
            stride = 1
            for a in range(dim):
                flat += pos[a] * stride
                stride *= n
            nodes.append(flat)
        N = E.size
        dofs = [comp * N + nodes[c] for c in range(nloc) for comp in range(dim)]
        sub = K[np.ix_(dofs, dofs)]
        assert np.abs(sub - 3.7 * Ke).max() <= 1e-12 * np.abs(Ke).max()
        mask = np.ones(K.shape, bool)
        mask[np.ix_(dofs, dofs)] = False
        assert np.abs(K[mask]).max() == 0.0


# -------------------------------------------------------------------- P4 --
@pytest.mark.parametrize("shape", [(8, 6), (4, 6, 8)])
def test_p4_operator_probes(shape):
    """K symmetric PSD with constants in its kernel (Sec. 2.3); M^-1 symmetric
    PSD; G K_ref = I - mean (pseudo-inverse, Sec. 3.1); G 1 = 0 (Sec. 5)."""
    rng = np.random.default_rng(1)
    dim = len(shape)
    E = ji.uniform_random_field(shape, 1.0, 1e3, seed=2)
    x = rng.standard_normal((dim,) + shape)
    y = rng.standard_normal((dim,) + shape)
    Kx = oracle.stiffness(E, x, LAM, MU)
    Ky = oracle.stiffness(E, y, LAM, MU)
    knorm = np.abs(Kx).max() / np.abs(x).max() * 10
    nx, ny = np.linalg.norm(x), np.linalg.norm(y)
    assert abs((y * Kx).sum() - (x * Ky).sum()) <= 1e-13 * knorm * nx * ny
    assert (x * Kx).sum() >= -1e-13 * knorm * nx * nx
    for a in range(dim):
        one = np.zeros((dim,) + shape)
        one[a] = 1.0
        assert np.abs(oracle.stiffness(E, one, LAM, MU)).max() <= 1e-12 * knorm
    G = oracle.green(shape, LAM, MU)
    diag, _ = oracle.jacobi_diag(E, LAM, MU)
    for pc in (oracle.PC_GREEN, oracle.PC_GREEN_JACOBI, oracle.PC_JACOBI):
        Mx, ratio = oracle.precond(pc, x, diag=diag, G=G)
        My, _ = oracle.precond(pc, y, diag=diag, G=G)
        mnorm = np.abs(Mx).max() / np.abs(x).max() * 10
        assert abs((y * Mx).sum() - (x * My).sum()) <= 1e-12 * mnorm * nx * ny
        assert (x * Mx).sum() >= -1e-13 * mnorm * nx * nx
        assert ratio <= 1e-12
    # Green: G K_ref v = v - mean(v), G 1 = 0
    Kref_x = oracle.stiffness(np.ones(shape), x, LAM, MU)
    GKx, _ = oracle.precond(oracle.PC_GREEN, Kref_x, G=G)
    xm = x - x.mean(axis=tuple(range(1, dim + 1)), keepdims=True)
    assert np.abs(GKx - xm).max() <= 1e-12 * np.abs(x).max()
    for a in range(dim):
        one = np.zeros((dim,) + shape)
        one[a] = 1.0
        z, _ = oracle.precond(oracle.PC_GREEN, one, G=G)
        assert np.abs(z).max() <= 1e-14


# -------------------------------------------------------------------- P6 --
@pytest.mark.parametrize("shape", [(4, 4), (6, 8), (4, 4, 4), (4, 6, 8)])
def test_p6_alg2_diagonal(shape):
    """Algorithm 2 uses d 2^d applications (8 in 2D, 24 in 3D; Sec. 3.3) and
    gives the diagonal of K: the closed-form box sum
    diag_a(I) = sum_{e containing I} E_e [(lam + 2 mu) I_a + mu sum_{b != a} I_b],
    I_a = int_e (d_a phi)^2 = prod_{b != a}(h_b / 3) / h_a (k_2 = (lam + 3 mu)/3 and
    k_3 = h (lam + 4 mu)/9 on square/cubic pixels), and (on 4^d) the diagonal of
    the dense matrix."""
    dim = len(shape)
    E = ji.uniform_random_field(shape, 1.0, 1e4, seed=3)
    diag, napply = oracle.jacobi_diag(E, LAM, MU)
    gold = golden()
    assert napply == int(gold[f"alg2_applications_{dim}d"][0]) == dim * 2 ** dim
    box = np.zeros(shape)
    for off in np.ndindex(*(2,) * dim):
        box += np.roll(E, shift=off, axis=tuple(range(dim)))
    h = 1.0 / np.array(shape[::-1], dtype=float)  # (hx, hy[, hz])
    Ia = [np.prod([h[b] / 3 for b in range(dim) if b != a]) / h[a] for a in range(dim)]
    for a in range(dim):
        ka = (LAM + 2 * MU) * Ia[a] + MU * sum(Ia[b] for b in range(dim) if b != a)
        assert np.abs(diag[a] - ka * box).max() <= 1e-12 * np.abs(diag).max()
    if len(set(shape)) == 1:
        kd = (LAM + 3 * MU) / 3 if dim == 2 else h[0] * (LAM + 4 * MU) / 9
        assert np.abs(diag[0] - kd * box).max() <= 1e-12 * np.abs(diag).max()
    if E.size <= 64:
        K = dense_K(E, LAM, MU)
        assert np.abs(np.diag(K) - diag.ravel()).max() <= 1e-13 * np.abs(diag).max()


def test_alg2_rejects_odd_grid():
    with pytest.raises(RuntimeError, match="odd_grid"):
        oracle.jacobi_diag(np.ones((5, 4)), LAM, MU)


# -------------------------------------------------------------------- P1 --
@pytest.mark.parametrize("shape", [(8, 8), (4, 6, 4)])
def test_p1_homogeneous(shape):
    """Constant E: f = 0 (B^T W constant = 0), no iteration, zero
    fluctuation, sigma_bar = E C eps_bar and C_eff = E C."""
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    E = np.full(shape, 2.5)
    rng = np.random.default_rng(4)
    macro = rng.standard_normal(ds)
    f, fa = oracle.rhs(E, macro, LAM, MU, with_abs=True)
    assert np.linalg.norm(f) <= 1e-14 * np.linalg.norm(fa)
    res = oracle.solve(E, macro, LAM, MU, pc=oracle.PC_GREEN_JACOBI)
    assert res.iters == 0 and res.status == "ok"
    assert np.abs(res.u).max() == 0.0
    Cm = 2.5 * mandel_iso(dim, LAM, MU)
    assert np.abs(res.sigma_bar - Cm @ macro).max() <= 1e-14 * np.abs(Cm @ macro).max()


# -------------------------------------------------------------------- P2 --
def laminate_sigma_bar(Ecols, dim, lam, mu, macro):
    """Exact homogenised stress of a layered medium with normal e_1 and equal
    layer widths: continuity of traction sigma e_1 and of u, zero average jump."""
    ds = dim * (dim + 1) // 2
    Nm = np.zeros((ds, dim))
    Nm[0, 0] = 1.0
    if dim == 2:
        Nm[2, 1] = 1 / np.sqrt(2)
    else:
        Nm[5, 1] = 1 / np.sqrt(2)
        Nm[4, 2] = 1 / np.sqrt(2)
    Cs = [E * mandel_iso(dim, lam, mu) for E in Ecols]
    A = [Nm.T @ Ck @ Nm for Ck in Cs]
    t0 = [Nm.T @ Ck @ macro for Ck in Cs]
    Ainv = [np.linalg.inv(a) for a in A]
    t = np.linalg.solve(np.mean(Ainv, axis=0), np.mean([ai @ tk for ai, tk in zip(Ainv, t0)], axis=0))
    sig = [Ck @ (macro + Nm @ (ai @ (t - tk))) for Ck, ai, tk in zip(Cs, Ainv, t0)]
    return np.mean(sig, axis=0)


@pytest.mark.parametrize("shape,chi", [((8, 16), 1e4), ((4, 4, 8), 10.0), ((6, 4, 8), 1e3)])
def test_p2_laminate_closed_form(shape, chi):
    """Laminate of Sec. 4.1: the exact fluctuation is piecewise linear in x_1
    and lies in the Q1 space, so sigma_bar equals the layered formula."""
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    E = ji.laminate_field(shape, chi)
    rng = np.random.default_rng(5)
    macro = rng.standard_normal(ds)
    res = oracle.solve(E, macro, LAM, MU, pc=oracle.PC_GREEN_JACOBI, tol=1e-13, maxit=3000)
    assert res.status == "ok"
    expect = laminate_sigma_bar(E.reshape(-1, shape[-1])[0], dim, LAM, MU, macro)
    assert np.abs(res.sigma_bar - expect).max() <= 1e-10 * np.abs(expect).max()


# -------------------------------------------------------------------- P3 --
@pytest.mark.parametrize("shape", [(8, 6), (8, 8), (4, 6, 8), (6, 6, 6)])
def test_p3_one_iteration(shape):
    """Constant C = s C_ref: G = K^+ up to 1/s (Sec. 3.1), so PCG converges in
    one iteration with Green.  On square/cubic pixels diag(K) is the same for
    every dof, J is a multiple of I and Green-Jacobi also needs one; on
    rectangular pixels the components get different diagonals and it does not."""
    dim = len(shape)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((dim,) + shape)
    f -= f.mean(axis=tuple(range(1, dim + 1)), keepdims=True)
    E = np.full(shape, 7.0)
    pcs = [oracle.PC_GREEN]
    if len(set(shape)) == 1:
        pcs.append(oracle.PC_GREEN_JACOBI)
    for pc in pcs:
        res = oracle.solve(E, np.zeros(dim * (dim + 1) // 2), LAM, MU, pc=pc, tol=1e-12, f=f,
                           hist_len=4)
        assert res.iters == 1, (pc, res.iters)
        assert res.relres <= 1e-13


# -------------------------------------------------------------------- P5 --
@pytest.mark.parametrize("shape", [(4, 4), (4, 4, 4)])
def test_p5_dense_direct(shape):
    """PCG result equals the dense bordered solve [K 1; 1^T 0] (unique
    mean-free solution, Sec. 2 space V)."""
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    E = ji.uniform_random_field(shape, 1.0, 1e4, seed=7)
    macro = np.arange(1, ds + 1, dtype=float) / ds
    K = dense_K(E, LAM, MU)
    f = oracle.rhs(E, macro, LAM, MU).ravel()
    N = E.size
    ndof = dim * N
    border = np.zeros((ndof, dim))
    for a in range(dim):
        border[a * N:(a + 1) * N, a] = 1.0
    A = np.block([[K, border], [border.T, np.zeros((dim, dim))]])
    sol = np.linalg.solve(A, np.concatenate([f, np.zeros(dim)]))[:ndof]
    for pc in (oracle.PC_GREEN, oracle.PC_GREEN_JACOBI, oracle.PC_JACOBI, oracle.PC_NONE):
        res = oracle.solve(E, macro, LAM, MU, pc=pc, tol=1e-14, maxit=5000)
        err = np.linalg.norm(res.u.ravel() - sol) / np.linalg.norm(sol)
        assert err <= 1e-10, (pc, err, res.status)


def test_cg_krylov_distinct_eigenvalues():
    """Unpreconditioned CG on uniform E terminates in at most as many steps as
    K has distinct nonzero eigenvalues (the Fourier symbol's eigenvalues)."""
    shape = (4, 4)
    rng = np.random.default_rng(8)
    f = rng.standard_normal((2,) + shape)
    f -= f.mean(axis=(1, 2), keepdims=True)
    Kc = symbol_closed_form(shape, LAM, MU)
    ev = np.linalg.eigvalsh(np.moveaxis(Kc.reshape(2, 2, -1), -1, 0)[1:]).ravel()
    distinct = len(np.unique(np.round(ev / ev.max(), 10)))
    res = oracle.solve(np.ones(shape), np.zeros(3), LAM, MU, pc=oracle.PC_NONE, tol=1e-12,
                       f=f, maxit=100)
    assert res.status == "ok"
    assert res.iters <= distinct


# ----------------------------------------------------------------- P8/P9 --
def test_p8_p9_hill_mandel_and_bounds():
    """Hill-Mandel: eps_bar . sigma_bar = <eps . sigma> (B^T W sigma = 0 at
    equilibrium, eq. non_lin_system); C_eff symmetric and between the Reuss
    and Voigt bounds (conforming FE)."""
    shape = (6, 6, 6)
    E = ji.grf_field(shape, 1e3, seed=1, ell=0.2)
    dim = 3
    rng = np.random.default_rng(9)
    macro = rng.standard_normal(6)
    res = oracle.solve(E, macro, LAM, MU, tol=1e-12, maxit=2000)
    sbar, sq = oracle.stress(E, macro, res.u, LAM, MU, want_field=True)
    # strains at the quadrature points: stress with the identity Mandel tensor
    # (lam = 0, mu = 1/2) and unit modulus
    _, eq = oracle.stress(np.ones(shape), macro, res.u, 0.0, 0.5, want_field=True)
    w = 1.0 / E.size / 8
    assert abs(macro @ sbar - w * (eq * sq).sum()) <= 1e-9 * abs(macro @ sbar)
    Ceff, _ = oracle.effective_stiffness(E, LAM, MU, tol=1e-12)
    assert np.abs(Ceff - Ceff.T).max() <= 1e-8 * np.abs(Ceff).max()
    Cm = mandel_iso(dim, LAM, MU)
    voigt = E.mean() * Cm
    reuss = np.linalg.inv((1.0 / E).mean() * np.linalg.inv(Cm))
    sym = 0.5 * (Ceff + Ceff.T)
    assert np.linalg.eigvalsh(voigt - sym).min() >= -1e-9 * np.abs(voigt).max()
    assert np.linalg.eigvalsh(sym - reuss).min() >= -1e-9 * np.abs(voigt).max()


# --------------------------------------------------------------- P10/P11 --
def test_p10_p11_preconditioner_independence_and_mean_shift():
    """All preconditioners give the same mean-free solution (Sec. 5); Green
    iterates are mean-free while Green-Jacobi iterates carry a mean that the
    outer J^1/2 introduces (Sec. 5, explanation)."""
    shape = (16, 16)
    # no reflection symmetry (a symmetric field would force zero means)
    E = ji.grf_field(shape, 1e3, seed=0, ell=0.2)
    macro = np.array([1.0, 0.0, 0.0])
    sols = {}
    for pc in (oracle.PC_NONE, oracle.PC_GREEN, oracle.PC_JACOBI, oracle.PC_GREEN_JACOBI):
        res = oracle.solve(E, macro, LAM, MU, pc=pc, tol=1e-12, maxit=20000, remove_mean=False)
        assert res.status == "ok"
        sols[pc] = res
    g = sols[oracle.PC_GREEN].u
    gj = sols[oracle.PC_GREEN_JACOBI].u
    assert np.abs(g.mean(axis=(1, 2))).max() <= 1e-11 * np.abs(g).max()
    assert np.abs(gj.mean(axis=(1, 2))).max() >= 1e-6 * np.abs(gj).max()
    ref = g - g.mean(axis=(1, 2), keepdims=True)
    for pc, res in sols.items():
        u = res.u - res.u.mean(axis=(1, 2), keepdims=True)
        assert np.linalg.norm(u - ref) <= 1e-8 * np.linalg.norm(ref), pc
        assert np.abs(res.sigma_bar - sols[oracle.PC_GREEN].sigma_bar).max() <= 1e-10


# ------------------------------------------------------------------- P12 --
def test_p12_scale_invariance():
    """E -> s E leaves u and the iteration count unchanged and scales sigma_bar
    (C_ref and J enter PCG only up to scalar factors)."""
    E = ji.sine_contrast_field(16)
    macro = np.array([0.3, -1.0, 0.5])
    a = oracle.solve(E, macro, LAM, MU, tol=1e-10, hist_len=100)
    b = oracle.solve(8.0 * E, macro, LAM, MU, tol=1e-10, hist_len=100)
    c = oracle.solve(E, macro, LAM, MU, lam_ref=3 * LAM, mu_ref=3 * MU, tol=1e-10, hist_len=100)
    # identical iterates up to rounding; the stop may flip by one at the boundary
    assert abs(a.iters - b.iters) <= 1 and abs(a.iters - c.iters) <= 1
    # late recursive residuals are dominated by cancellation (relative error
    # ~ eps ||r_0|| / ||r_k||); compare the part of the history above 1e-5 ||r_0||
    r0 = np.linalg.norm(oracle.rhs(E, macro, LAM, MU))
    m = int(np.sum(a.res > 1e-5 * r0))
    assert m >= 5
    assert np.abs(b.res[:m] / 8.0 / a.res[:m] - 1).max() <= 1e-8
    assert np.abs(c.res[:m] / a.res[:m] - 1).max() <= 1e-8
    assert np.abs(b.alpha[:m] / a.alpha[:m] - 1).max() <= 1e-8  # K x8, M^-1 x1/8
    assert np.abs(c.alpha[:m] / 3.0 / a.alpha[:m] - 1).max() <= 1e-8  # G x1/3, p x1/3
    assert np.linalg.norm(a.u - b.u) <= 1e-9 * np.linalg.norm(a.u)
    assert np.linalg.norm(a.u - c.u) <= 1e-9 * np.linalg.norm(a.u)
    assert np.abs(8.0 * a.sigma_bar - b.sigma_bar).max() <= 1e-9 * np.abs(b.sigma_bar).max()


# ------------------------------------------------------------------- P13 --
def test_p13_void_replacement_value():
    """Zero diagonal entries replaced by any value leave the iteration count
    unchanged (Sec. 3.2); cosine geometry with chi = infinity (Sec. 4.2) and a
    block of void pixels that creates exact zero diagonal entries."""
    gold = golden()["void_values"] + [1.0]
    fields = []
    fields.append(ji.cosine_void_field(16, None))
    E = ji.cosine_void_field(16, 1e4)
    E[4:9, 4:9] = 0.0
    fields.append(E)
    for E in fields:
        diag, _ = oracle.jacobi_diag(E, LAM, MU)
        counts = []
        for v in gold:
            res = oracle.solve(E, np.array([1.0, 1.0, 1.0]), LAM, MU, pc=oracle.PC_GREEN_JACOBI,
                               tol=1e-8, maxit=5000, void_value=v)
            assert res.status == "ok"
            counts.append(res.iters)
        assert len(set(counts)) == 1, counts
    assert (diag == 0).sum() > 0


# ------------------------------------------------------------ constants --
def test_paper_reference_material_constants():
    """lambda^0 = 2/3, mu^0 = 1/2 give bulk modulus K^0 = 1 (Sec. 4)."""
    g = golden()
    lam0, mu0 = g["lame_lambda0"][0], g["lame_mu0"][0]
    assert abs(lam0 + 2 * mu0 / 3 - g["bulk_modulus_K0"][0]) <= 1e-15
    Cm = mandel_iso(3, lam0, mu0)
    # bulk response: sigma_kk / (3 eps_kk) for eps = I/3
    eps = np.array([1, 1, 1, 0, 0, 0]) / 3
    assert abs((Cm @ eps)[:3].sum() / 3 - 1.0) <= 1e-15


def test_stiffness_at_node_matches_full():
    shape = (6, 4, 8)
    E = ji.uniform_random_field(shape, 1, 10, seed=10)
    u = np.random.default_rng(11).standard_normal((3,) + shape)
    full = oracle.stiffness(E, u, LAM, MU).reshape(3, -1)
    for node in [0, 5, 77, E.size - 1]:
        assert np.abs(oracle.stiffness_at_node(E, u, LAM, MU, node) - full[:, node]).max() <= 1e-13 * np.abs(full).max()


def test_trend_green_vs_green_jacobi_sine_contrast_32x32():
    """Smooth contrast-1e4 field on 32^2 (Sec. 1 / Sec. 6 trend): Green-Jacobi
    needs fewer iterations than Green.  Reported, and checked as a trend."""
    E = ji.sine_contrast_field(32)
    g = oracle.solve(E, np.array([1.0, 0, 0]), LAM, MU, pc=oracle.PC_GREEN, tol=1e-8, maxit=5000)
    gj = oracle.solve(E, np.array([1.0, 0, 0]), LAM, MU, pc=oracle.PC_GREEN_JACOBI, tol=1e-8)
    assert gj.iters < g.iters


# ------------------------------------------------- rounding-difference models
def test_dot2_matches_correctly_rounded_sum():
    """Dot2 (Ogita, Rump, Oishi 2005) is as accurate as a sum in twice the
    working precision: on ill-conditioned dot products (the terms cancel to
    one part in ~1e16) it agrees with the exact dot product (rational
    arithmetic, then rounded) to a few ulps, where the serial sum loses
    digits."""
    from fractions import Fraction
    rng = np.random.default_rng(5)
    worst_serial = 0.0
    for trial in range(10):
        n = 300
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-8, 8, n)
        y = rng.standard_normal(n)
        x = np.concatenate([x, -x * (1 + 2.0 ** -40), [1e-3]])
        y = np.concatenate([y, y, [1.0]])
        exact = float(sum(Fraction(a) * Fraction(b) for a, b in zip(x, y)))
        d2 = oracle.dot(x, y, mode=1)
        assert abs(d2 - exact) <= 4 * 2.0 ** -52 * abs(exact), (trial, d2, exact)
        worst_serial = max(worst_serial, abs(oracle.dot(x, y, mode=0) - exact) / abs(exact))
    assert worst_serial > 1e-6  # the serial sum does lose digits on these
    # the plain dot is the serial sum in index order
    a = rng.standard_normal(1000)
    b = rng.standard_normal(1000)
    s = 0.0
    for u, v in zip(a, b):
        s += u * v
    assert oracle.dot(a, b, mode=0) == s


def test_rounding_models_keep_the_solution():
    """The parity-window options change rounding only: with Dot2 inner
    products or one-ulp noise on every K p and M^-1 r result the solve
    reaches the same solution (to the tolerance) and the early CG scalars
    agree to rounding; the noisy run's scalars differ from the plain run's
    (the noise is on); noise_seed = 0 with dot_mode = 0 is the plain
    arithmetic bit for bit."""
    E = ji.sine_contrast_field(32)
    m = np.array([1.0, 0.0, 0.0])
    base = oracle.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=500, hist_len=100)
    for kw in (dict(dot_mode=1), dict(noise_seed=7), dict(noise_seed=7, dot_mode=1)):
        r = oracle.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=500, hist_len=100, **kw)
        assert r.status == "ok"
        assert np.linalg.norm(r.u - base.u) <= 1e-10 * np.linalg.norm(base.u)
        assert np.abs(r.alpha[:3] / base.alpha[:3] - 1).max() <= 1e-12
        assert abs(r.iters - base.iters) <= 2
        if "noise_seed" in kw:
            assert not np.array_equal(r.alpha[:5], base.alpha[:5])
    again = oracle.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=500, hist_len=100, noise_seed=0,
                         dot_mode=0)
    assert np.array_equal(again.u, base.u) and np.array_equal(again.alpha, base.alpha)


def test_triangle_and_powerlaw_rounding_models():
    """The same options in the numpy oracles: a Dot2-like (math.fsum) or noisy
    triangle solve reaches the plain solution; a noisy power-law PCG solve
    reaches the plain one."""
    from oracle import triangles as tri
    E = ji.sine_contrast_field(16)
    m = np.array([1.0, 0.0, 0.0])
    base = tri.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=500)
    for kw in (dict(dot_mode=1), dict(noise_seed=3)):
        r = tri.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=500, **kw)
        assert r.status == "ok" and abs(r.iters - base.iters) <= 2
        assert np.linalg.norm(r.u - base.u) <= 1e-10 * np.linalg.norm(base.u)


def test_precond_fft_equals_naive_dft_precond():
    """oracle.precond_fft (numpy's FFT as the transform step) is the same
    operator as the naive-DFT precond: agreement to 1e-13 for the four
    preconditioners, 2D and 3D, with a void."""
    rng = np.random.default_rng(9)
    for shape in ((12, 10), (6, 8, 4)):
        dim = len(shape)
        E = ji.uniform_random_field(shape, 1.0, 1e3, seed=2)
        E.flat[3] = 0.0
        dg, _ = oracle.jacobi_diag(E, LAM, MU)
        G = oracle.green(shape, LAM, MU)
        r = rng.standard_normal((dim,) + shape)
        for pc in (0, 1, 2, 3):
            z, _ = oracle.precond(pc, r, diag=dg, G=G, void_value=2.0)
            zf = oracle.precond_fft(pc, r, diag=dg, G=G, void_value=2.0)
            assert np.abs(z - zf).max() <= 1e-13 * np.abs(z).max(), (shape, pc)


def test_python_loop_equals_c_loop():
    """oracle.solve_py follows or_solve's loop: with the naive DFT its early
    CG scalars equal the C loop's to rounding, and both (and the FFT
    variant) reach the same solution and sigma_bar; the iteration counts
    agree within a few iterations (summation order only)."""
    E = ji.grf_field((12, 10, 8), 1e3, seed=4)
    m = np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    c = oracle.solve(E, m, LAM, MU, pc=3, tol=1e-12, maxit=2000, hist_len=50)
    for tr in ("dft", "fft"):
        p = oracle.solve_py(E, m, LAM, MU, pc=3, tol=1e-12, maxit=2000, hist_len=50,
                            transform=tr)
        assert p.status == "ok"
        assert abs(p.iters - c.iters) <= 3
        assert np.abs(p.alpha[:5] / c.alpha[:5] - 1).max() <= 1e-12
        assert np.linalg.norm(p.u - c.u) <= 1e-10 * np.linalg.norm(c.u)
        assert np.abs(p.sigma_bar - c.sigma_bar).max() <= 1e-11 * np.abs(c.sigma_bar).max()
    # homogeneous material: zero iterations, u = 0
    h = oracle.solve_py(np.full((6, 4), 2.0), np.array([1.0, 0.5, 0.2]), LAM, MU, pc=3)
    assert h.iters == 0 and np.abs(h.u).max() == 0.0

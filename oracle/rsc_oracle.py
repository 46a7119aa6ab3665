"""Plain FP64 CPU reference for rotational OMP in a steerable circular-harmonic basis.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls this
module; only the tests, the smoke check and the CPU-baseline timing of the
benchmark do.  It is written to be checked against the paper by eye: no
factoring, no blocking, a dense augmented dictionary and a fresh QR
least-squares solve at every pursuit step.

Paper: McCann, Andrearczyk, Unser, Depeursinge, "Fast Rotational Sparse Coding"
(arXiv 1806.04374).  Section and equation numbers below refer to it:
  eq. (2)  rotational sparse coding objective (Sec. II-B)
  eq. (3)  rotation covariance of the code (Sec. II-B)
  eq. (4)  rearrangement with a unitary steerable basis (Sec. II-D)
  eq. (5)  annular circular-harmonic basis functions (Sec. II-D)
  eq. (6)  rotation multiplies harmonic t by exp(-i t theta0) (Sec. II-D)
  eq. (7)  sampling on the grid, normalisation, column stacking (Sec. II-D)
  eq. (8)  steering matrix S_r (Sec. II-D)
  Sec. II-C and Fig. 2 (pseudocode): augmented dictionary [R_0 D ... R_{R-1} D]
           and OMP over it.
  Sec. II-E  proposed algorithm: basis, hat coordinates, R-K-SVD with S_r in
           place of R_r, back to pixels with Phi.

Readings where the paper is silent:
  * Grid axes: pixel (row i, col j) sits at x = j - c, y = c - i (y up),
    c = (N-1)/2; angles are atan2(y, x), counter-clockwise.
  * Disk: pixels with radius < N/2 (97 pixels at N = 11, as printed in III-A).
  * Radial profiles are Gaussian windows exp(-(rho - rho_s)^2 / (2 sigma^2))
    with rho_s = s (N/2)/S, s = 1..S and sigma = (N/2)/S, in place of the
    annulus indicator of eq. (5).  Every harmonic k = 0..T is kept on every
    profile.  The centre pixel is set to 0 for k != 0 (its angle is undefined).
  * After the per-column normalisation of eq. (7), the S columns of each
    harmonic are Loewdin-orthonormalised (Phi_k <- Phi_k G_k^{-1/2}); this
    keeps the columns of a harmonic orthogonal, as the disjoint annuli of
    eq. (5) are, and does not change the span or steerability.
  * Packed real coordinates, harmonic-major: [k=0: s=0..S-1], then for each
    k = 1..T [Re: s=0..S-1][Im: s=0..S-1].  The real synthesis vectors are
    Re phi_{s,0}, sqrt(2) Re phi_{s,k} and -sqrt(2) Im phi_{s,k}; a packed pair
    (a, b) stands for the complex coefficient (a + i b)/sqrt(2) on phi_{s,k}
    and its conjugate on phi_{s,-k}.
  * Steering by r multiplies (a + i b) of harmonic k by exp(-i k 2 pi r / R),
    the sign of eq. (6)/(8).
  * Pursuit: select the column of largest |correlation|; exact ties go to the
    smallest atom index, then the smallest angle index; stop early when
    ||r||^2 <= tau^2 ||x||^2 (tau = 1e-5) or when the selected column is
    already in the support.  The same atom at another angle may be selected
    (Sec. II-B).  Empty slots are (-1, -1, 0).
  * Dictionary update (R-K-SVD, Fig. 2 and Sec. II-C), in hat coordinates
    (Sec. II-E): the augmented dictionary is built once per outer iteration, so
    every atom is updated from the same codes and the same old dictionary.  When
    a patch uses atom m more than once, r0 is the angle of the first such slot in
    selection order.  The first singular vector's sign is chosen to agree with
    the old atom (<d_new, d_old> > 0; when that is 0, the largest-magnitude
    coordinate is made positive, the first one on ties).  Atoms that no patch
    uses are reset, in increasing index, to the directions of the patches with
    the largest current coding error ||x_p - D a_p||^2, one distinct patch each,
    in decreasing order of that error (ties: smaller patch index); only patches
    with a positive error qualify, and an unused atom keeps its value when none
    is left.  After the last iteration the pursuit runs once more so that the
    codes belong to the final dictionary.
  * Texture classifier (Sec. III-B, "Classifier"): a patch's "sum squared error"
    under a class dictionary is the pursuit's own squared residual in hat
    coordinates, ||x_hat - D_aug b||^2 (what the coder minimises; in pixels it
    differs by a class-independent term and the basis Gram weighting).  Label =
    the class of smallest error, ties to the smaller class index.  An image's
    feature is its label histogram normalised to frequencies (the paper's images
    all have one size, where counts and frequencies rank neighbours alike).
    chi^2 terms with a[i] + b[i] = 0 are 0.  The nearest neighbour's ties go to
    the smaller training index.
  * The paper's own annular basis (eq. (5)-(7), Sec. II-D) for rotation: S = floor(N/2)
    annuli N(s-1)/(2S) <= r < N s/(2S); harmonics -T_s..T_s on annulus s with T_s the
    half circumference floor(pi r_mid) (r_mid the annulus' middle radius, which gives the
    (1, 5, 8) of the paper's basis figure at N = 11), lowered where needed to the largest
    value whose 2 T_s + 1 harmonic columns are linearly independent on the annulus' pixels
    (taken as it is, the rule asks the 8-pixel second annulus at N = 11 for 11 columns,
    and (Phi^* Phi)^{-1} would not exist).  The low-pass basis halves these T_s (floor).
    The centre pixel is 0 for t != 0, as above; columns are normalised and need no
    orthonormalisation (annuli are disjoint).  Packed real coordinates as above,
    harmonic-major, with the annuli whose T_s >= k in each harmonic-k block.  The pursuit
    on it is the same OMP over [S_0 D, ..., S_{R-1} D], with the steering of that ragged
    layout (harmonic k of each of its annuli multiplied by exp(-i k theta)).
  * Rotation by interpolation (Sec. III-C, rotation speed): rotating a patch by theta
    (counter-clockwise, about its centre pixel) sets output pixel (x, y) to the input
    at R_{-theta}(x, y), read with nearest-neighbour interpolation (coordinates
    rounded half up) or bicubic interpolation (Keys' cubic convolution, a = -1/2, over
    the 4 x 4 neighbours); input pixels outside the N x N patch count as 0.
"""
from __future__ import annotations

import dataclasses

import numpy as np

TAU = 1e-5


# --------------------------------------------------------------------------- grid
def disk_grid(N: int):
    """Grid of eq. (7) restricted to the circular patch of Sec. III-A.

    Returns (mask [N,N] bool, rho, theta) with rho/theta of the disk pixels in
    row-major order.  x = col - c, y = c - row, theta = atan2(y, x).
    """
    if N < 1 or N % 2 == 0:
        raise ValueError("N must be odd and positive")
    c = (N - 1) / 2
    rows, cols = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x = cols - c
    y = c - rows
    rho = np.sqrt(x * x + y * y)
    mask = rho < N / 2
    return mask, rho[mask], np.arctan2(y[mask], x[mask])


def default_profiles(N: int, S: int):
    """Gaussian profile centres rho_s = s (N/2)/S (s = 1..S) and width sigma = (N/2)/S."""
    sigma = (N / 2) / S
    return sigma * np.arange(1, S + 1, dtype=np.float64), sigma


@dataclasses.dataclass
class Basis:
    N: int
    S: int
    T: int
    mask: np.ndarray          # [N, N] disk
    phi_c: np.ndarray         # [T+1, S, n_pix] complex columns phi_{s,k}, k >= 0
    phi: np.ndarray           # [n_pix, B] packed real synthesis matrix
    pinv: np.ndarray          # [B, n_pix] (Phi^T Phi)^{-1} Phi^T

    @property
    def B(self) -> int:
        return self.S * (2 * self.T + 1)

    @property
    def n_pix(self) -> int:
        return int(self.mask.sum())


def build_basis(N: int, S: int, T: int, centres=None, sigma=None) -> Basis:
    """Discrete steerable basis, eq. (5)-(7), with the Gaussian-profile reading above."""
    mask, rho, theta = disk_grid(N)
    if centres is None or sigma is None:
        centres, sigma = default_profiles(N, S)
    centres = np.asarray(centres, dtype=np.float64)
    n = rho.size
    phi_c = np.zeros((T + 1, S, n), dtype=np.complex128)
    for k in range(T + 1):
        for s in range(S):
            col = np.exp(-((rho - centres[s]) ** 2) / (2.0 * sigma * sigma)) * np.exp(1j * k * theta)
            if k != 0:
                col[rho == 0] = 0.0
            phi_c[k, s] = col / np.linalg.norm(col)
        # Loewdin orthonormalisation of the S columns of harmonic k
        cols = phi_c[k].T                                 # [n, S]
        gram = cols.conj().T @ cols                       # [S, S] Hermitian
        w, v = np.linalg.eigh(gram)
        inv_sqrt = (v / np.sqrt(w)) @ v.conj().T
        phi_c[k] = (cols @ inv_sqrt).T
    # packed real synthesis vectors, harmonic-major
    blocks = [phi_c[0].real.T]
    for k in range(1, T + 1):
        blocks.append(np.sqrt(2.0) * phi_c[k].real.T)
        blocks.append(-np.sqrt(2.0) * phi_c[k].imag.T)
    phi = np.concatenate(blocks, axis=1)                  # [n, B]
    # biorthogonal partner (Phi^T Phi)^{-1} Phi^T, Sec. II-D
    pinv = np.linalg.solve(phi.T @ phi, phi.T)
    return Basis(N, S, T, mask, phi_c, phi, pinv)


# --------------------------------------------------------------------------- annular basis
def _annulus_columns(rho: np.ndarray, theta: np.ndarray, T: int) -> np.ndarray:
    """Complex columns exp(i t theta), t = -T..T, on the given pixels (eq. (5)); the centre
    pixel (rho = 0) is 0 for t != 0."""
    t = np.arange(-T, T + 1)
    A = np.exp(1j * np.outer(theta, t))
    A[(rho == 0)[:, None] & (t != 0)[None, :]] = 0.0
    return A


def annular_cutoffs(N: int, lowpass: bool = False, cap: bool = True) -> list:
    """Per-annulus cut-offs T_s, s = 1..floor(N/2) (Sec. II-D): half the circumference,
    floor(pi r_mid); with cap, lowered to the largest T whose columns t = -T..T are linearly
    independent on the annulus (smallest singular value above 1e-6 of the largest); the
    low-pass basis halves them (Sec. III-C)."""
    S = N // 2
    _, rho, theta = disk_grid(N)
    out = []
    for s in range(1, S + 1):
        lo, hi = N * (s - 1) / (2 * S), N * s / (2 * S)
        ring = (rho >= lo) & (rho < hi)
        half = int(np.floor(np.pi * (lo + hi) / 2))
        T = half
        if cap:
            T = -1
            for t in range(half + 1):
                A = _annulus_columns(rho[ring], theta[ring], t)
                if A.shape[1] > A.shape[0]:
                    break
                sv = np.linalg.svd(A, compute_uv=False)
                if sv[-1] <= 1e-6 * sv[0]:
                    break
                T = t
        out.append(T // 2 if lowpass else T)
    return out


@dataclasses.dataclass
class AnnularBasis:
    N: int
    Ts: list                  # cut-off of annulus s = 1..S
    mask: np.ndarray          # [N, N] disk
    phi: np.ndarray           # [n_pix, B] packed real synthesis matrix
    pinv: np.ndarray          # [B, n_pix] (Phi^T Phi)^{-1} Phi^T

    @property
    def S(self) -> int:
        return len(self.Ts)

    @property
    def T(self) -> int:
        return max(self.Ts)

    @property
    def Sk(self) -> list:
        """Number of annuli carrying harmonic k, k = 0..T."""
        return [sum(1 for t in self.Ts if t >= k) for k in range(self.T + 1)]

    @property
    def B(self) -> int:
        return self.phi.shape[1]

    @property
    def n_pix(self) -> int:
        return int(self.mask.sum())


def build_annular_basis(N: int, lowpass: bool = False) -> AnnularBasis:
    """The paper's discrete steerable basis, eq. (5)-(7), with the cut-offs above."""
    mask, rho, theta = disk_grid(N)
    S = N // 2
    Ts = annular_cutoffs(N, lowpass)
    blocks = []
    for k in range(max(Ts) + 1):
        cols = []
        for s in range(1, S + 1):
            if Ts[s - 1] < k:
                continue
            lo, hi = N * (s - 1) / (2 * S), N * s / (2 * S)
            col = np.where((rho >= lo) & (rho < hi), np.exp(1j * k * theta), 0.0)
            if k != 0:
                col[rho == 0] = 0.0
            cols.append(col / np.linalg.norm(col))
        C = np.array(cols).T                                # [n_pix, annuli with T_s >= k]
        if k == 0:
            blocks.append(C.real)
        else:
            blocks.append(np.sqrt(2.0) * C.real)
            blocks.append(-np.sqrt(2.0) * C.imag)
    phi = np.concatenate(blocks, axis=1)
    pinv = np.linalg.solve(phi.T @ phi, phi.T)
    return AnnularBasis(N, Ts, mask, phi, pinv)


def steer_ragged(xhat: np.ndarray, theta, Sk: list) -> np.ndarray:
    """Steering (eq. (8)) in the harmonic-major layout with Sk[k] annuli in harmonic k:
    the complex coefficient (Re + i Im) of harmonic k is multiplied by exp(-i k theta)."""
    xhat = np.asarray(xhat, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    out = xhat.copy()
    off = Sk[0]
    for k in range(1, len(Sk)):
        n = Sk[k]
        re, im = slice(off, off + n), slice(off + n, off + 2 * n)
        z = (xhat[..., re] + 1j * xhat[..., im]) * np.exp(-1j * k * theta)[..., None]
        out[..., re] = z.real
        out[..., im] = z.imag
        off += 2 * n
    return out


def steer_basis(basis, xhat: np.ndarray, theta) -> np.ndarray:
    """Steering for either basis: the full (S, T) grid or the annular basis' ragged one."""
    if isinstance(basis, AnnularBasis):
        return steer_ragged(xhat, theta, basis.Sk)
    return steer(xhat, theta, basis.S, basis.T)


# --------------------------------------------------------------------------- coordinates
def project(basis: Basis, patches: np.ndarray) -> np.ndarray:
    """Hat coordinates x_hat = (Phi^* Phi)^{-1} Phi^* x (Sec. II-E, step 2).

    patches: [P, N, N]; pixels outside the disk are ignored.  Returns [P, B].
    Computed as a least-squares solve of Phi x_hat = x over the disk pixels.
    """
    X = np.asarray(patches, dtype=np.float64).reshape(len(patches), -1)
    Xd = X[:, basis.mask.ravel()]
    if Xd.shape[0] == 0:
        return np.zeros((0, basis.B))
    sol, *_ = np.linalg.lstsq(basis.phi, Xd.T, rcond=None)
    return sol.T


def to_pixels(basis: Basis, xhat: np.ndarray) -> np.ndarray:
    """Phi x_hat placed on the N x N grid, zero outside the disk (Sec. II-E, step 4)."""
    xhat = np.atleast_2d(xhat)
    out = np.zeros((xhat.shape[0], basis.N * basis.N))
    out[:, basis.mask.ravel()] = xhat @ basis.phi.T
    return out.reshape(-1, basis.N, basis.N)


def steer(xhat: np.ndarray, theta, S: int, T: int) -> np.ndarray:
    """Apply the steering matrix of eq. (8) for rotation angle theta (radians).

    Harmonic k of the complex coefficient is multiplied by exp(-i k theta);
    harmonic 0 is unchanged.  xhat [..., B]; theta broadcasts against xhat[..., 0].
    """
    xhat = np.asarray(xhat, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    out = xhat.copy()
    for k in range(1, T + 1):
        re = slice(S + 2 * S * (k - 1), S + 2 * S * (k - 1) + S)
        im = slice(S + 2 * S * (k - 1) + S, S + 2 * S * k)
        z = xhat[..., re] + 1j * xhat[..., im]
        z = z * np.exp(-1j * k * theta)[..., None]
        out[..., re] = z.real
        out[..., im] = z.imag
    return out


def augmented_dictionary(D_hat: np.ndarray, R: int, S: int, T: int) -> np.ndarray:
    """Dense augmented dictionary [S_0 D, S_1 D, ..., S_{R-1} D] (Fig. 2 with R_r -> S_r).

    Returned as rows: row j = r*M + m is S_r d_m, shape [M*R, B].
    """
    M = D_hat.shape[0]
    rows = np.empty((R * M, D_hat.shape[1]))
    for r in range(R):
        rows[r * M:(r + 1) * M] = steer(D_hat, 2 * np.pi * r / R, S, T)
    return rows


def augmented_dictionary_basis(basis, D_hat: np.ndarray, R: int) -> np.ndarray:
    """The augmented dictionary of Fig. 2 (R_r -> S_r) in the coordinate layout of either
    basis: the full (S, T) grid or the annular basis' harmonic-major blocks of Sk[k] annuli.
    Row j = r*M + m is S_r d_m, shape [M*R, B]."""
    M = D_hat.shape[0]
    rows = np.empty((R * M, D_hat.shape[1]))
    for r in range(R):
        rows[r * M:(r + 1) * M] = steer_basis(basis, D_hat, 2 * np.pi * r / R)
    return rows


# --------------------------------------------------------------------------- pursuit
@dataclasses.dataclass
class Code:
    atom: np.ndarray      # [P, K] int, -1 for empty slots
    angle: np.ndarray     # [P, K] int, -1 for empty slots
    coef: np.ndarray      # [P, K] float64, 0 for empty slots
    resid2: np.ndarray    # [P] squared hat-domain residual norm
    corr: np.ndarray      # [P, K] |correlation| of each selection (0 for empty)
    gap: np.ndarray       # [P, K] relative gap between the two largest |c| at each step


def _pick(absc: np.ndarray, M: int) -> int:
    """Largest |c|; exact ties go to the smallest atom index, then the smallest angle."""
    best = absc.max()
    cand = np.flatnonzero(absc == best)
    m = cand % M
    r = cand // M
    order = np.lexsort((r, m))
    return int(cand[order[0]])


def omp(D_aug: np.ndarray, xhat: np.ndarray, K: int, M: int, tau: float = TAU,
        trace=None) -> Code:
    """Orthogonal matching pursuit over the augmented dictionary (Sec. II-C).

    D_aug [M*R, B] rows are unit-norm columns of the augmented dictionary; xhat [P, B].
    Each step: correlate the residual with every column, take the largest
    magnitude, add it to the support, refit all coefficients on the support by
    least squares (Householder QR) and recompute the residual.
    ``trace(p, k, support, coef, residual)`` is called after each step when given.
    """
    xhat = np.asarray(xhat, dtype=np.float64)
    P = xhat.shape[0]
    atom = -np.ones((P, K), np.int64)
    angle = -np.ones((P, K), np.int64)
    coef = np.zeros((P, K))
    corr = np.zeros((P, K))
    gap = np.zeros((P, K))
    resid2 = np.zeros(P)
    res = xhat.copy()
    support = [[] for _ in range(P)]
    active = np.ones(P, dtype=bool)
    for k in range(K):
        for p in np.flatnonzero(active):
            if res[p] @ res[p] <= tau * tau * (xhat[p] @ xhat[p]):
                active[p] = False
        idx = np.flatnonzero(active)
        if idx.size == 0:
            break
        C = res[idx] @ D_aug.T                          # correlations of all columns
        for t, p in enumerate(idx):
            absc = np.abs(C[t])
            j = _pick(absc, M)
            if j in support[p]:
                active[p] = False
                continue
            support[p].append(j)
            A = D_aug[support[p]].T                     # [B, k+1]
            Q, Rm = np.linalg.qr(A)
            a = np.linalg.solve(Rm, Q.T @ xhat[p])
            res[p] = xhat[p] - A @ a
            corr[p, k] = absc[j]
            if absc.size > 1 and absc[j] > 0:
                second = np.partition(absc, -2)[-2]
                gap[p, k] = (absc[j] - second) / absc[j]
            if trace is not None:
                trace(p, k, list(support[p]), a.copy(), res[p].copy())
    for p in range(P):
        s = support[p]
        if s:
            A = D_aug[s].T
            Q, Rm = np.linalg.qr(A)
            a = np.linalg.solve(Rm, Q.T @ xhat[p])
            for i, j in enumerate(s):
                atom[p, i] = j % M
                angle[p, i] = j // M
                coef[p, i] = a[i]
        resid2[p] = res[p] @ res[p]
    return Code(atom, angle, coef, resid2, corr, gap)


def encode(basis: Basis, D_hat: np.ndarray, R: int, patches: np.ndarray, K: int,
           tau: float = TAU) -> tuple[np.ndarray, Code]:
    """Sec. II-E steps 2-3 for a fixed dictionary: hat coordinates, then OMP with S_r."""
    xhat = project(basis, patches)
    D_aug = augmented_dictionary_basis(basis, D_hat, R)
    return xhat, omp(D_aug, xhat, K, D_hat.shape[0], tau)


def code_to_hat(D_hat: np.ndarray, R: int, S: int, T: int, code: Code) -> np.ndarray:
    """sum_i a_i S_{r_i} d_{m_i} for each patch (empty slots contribute nothing)."""
    P, K = code.atom.shape
    out = np.zeros((P, D_hat.shape[1]))
    for p in range(P):
        for i in range(K):
            if code.atom[p, i] >= 0:
                out[p] += code.coef[p, i] * steer(D_hat[code.atom[p, i]],
                                                  2 * np.pi * code.angle[p, i] / R, S, T)
    return out


def code_to_hat_basis(basis, D_hat: np.ndarray, R: int, code: Code) -> np.ndarray:
    """code_to_hat in the coordinate layout of either basis."""
    P, K = code.atom.shape
    out = np.zeros((P, D_hat.shape[1]))
    for p in range(P):
        for i in range(K):
            if code.atom[p, i] >= 0:
                out[p] += code.coef[p, i] * steer_basis(basis, D_hat[code.atom[p, i]],
                                                        2 * np.pi * code.angle[p, i] / R)
    return out


def reconstruct(basis: Basis, D_hat: np.ndarray, R: int, code: Code) -> np.ndarray:
    """Pixel-domain reconstruction Phi sum_i a_i S_{r_i} d_{m_i} (Sec. II-E step 4), [P, N, N]."""
    return to_pixels(basis, code_to_hat_basis(basis, D_hat, R, code))


def mse(basis: Basis, patches: np.ndarray, recon: np.ndarray) -> float:
    """Mean over patches and disk pixels of the squared coding error (Sec. III-A metric)."""
    m = basis.mask
    d = (np.asarray(patches, np.float64) - recon)[:, m]
    return float(np.mean(d * d)) if d.size else 0.0


def span_error(basis: Basis, patches: np.ndarray) -> float:
    """Mean squared distance of the patches to span(Phi) on the disk (the lower bound of Sec. III-A)."""
    xhat = project(basis, patches)
    return mse(basis, patches, to_pixels(basis, xhat))


# --------------------------------------------------------------------------- synthesis
def synthesize(basis: Basis, D_hat: np.ndarray, atom, angle, weight, noise=None) -> np.ndarray:
    """Patches sum_i w_i Phi S_{theta_i} d_{m_i} (+ noise on all N x N pixels), [P, N, N]."""
    atom = np.asarray(atom)
    P, J = atom.shape
    hat = np.zeros((P, D_hat.shape[1]))
    for i in range(J):
        hat += np.asarray(weight)[:, i, None] * steer_basis(basis, D_hat[atom[:, i]], np.asarray(angle)[:, i])
    x = to_pixels(basis, hat)
    if noise is not None:
        x = x + noise
    return x


# --------------------------------------------------------------------------- images
def synthesize_image(basis: Basis, D_hat: np.ndarray, H: int, W: int, centre, atom, angle, amplitude,
                     noise=None) -> np.ndarray:
    """Texture image: sum of stamps amplitude * Phi S_theta d_m (an N x N patch, zero off the
    disk) whose centre pixel lands on integer position centre = (row, col), clipped at the
    borders, plus noise [H, W]."""
    N = basis.N
    c = (N - 1) // 2
    img = np.zeros((H, W))
    atom = np.asarray(atom)
    if atom.size:
        stamps = to_pixels(basis, np.asarray(amplitude)[:, None] *
                           steer(D_hat[atom], np.asarray(angle), basis.S, basis.T))
        for i in range(atom.size):
            r0, c0 = int(centre[i][0]) - c, int(centre[i][1]) - c
            ra, rb = max(r0, 0), min(r0 + N, H)
            ca, cb = max(c0, 0), min(c0 + N, W)
            if ra < rb and ca < cb:
                img[ra:rb, ca:cb] += stamps[i, ra - r0:rb - r0, ca - c0:cb - c0]
    if noise is not None:
        img = img + noise
    return img


def image_patches(img: np.ndarray, N: int) -> np.ndarray:
    """All stride-1 N x N windows of an image, origins in row-major order: [(H-N+1)(W-N+1), N, N]."""
    H, W = img.shape
    if H < N or W < N:
        return np.zeros((0, N, N))
    v = np.lib.stride_tricks.sliding_window_view(img, (N, N))
    return v.reshape(-1, N, N)


# --------------------------------------------------------------------------- dictionary update
def _sign_like(u: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """u or -u: the one with <u, ref> > 0; if <u, ref> = 0, the one whose
    largest-magnitude coordinate (the first on ties) is positive."""
    s = float(u @ ref)
    if s < 0 or (s == 0 and u[int(np.argmax(np.abs(u)))] < 0):
        return -u
    return u


def rksvd_update_basis(basis, D_hat: np.ndarray, R: int, xhat: np.ndarray, code: Code):
    """The atom update of rksvd_update in the coordinate layout of either basis (the full
    (S, T) grid or the annular basis of eq. (5)-(7)): the same steps, with that basis'
    steering S_r (Sec. II-E: the update runs in the steerable basis' coordinates)."""
    return _rksvd_update(D_hat, R, xhat, code, lambda v, th: steer_basis(basis, v, th))


def rksvd_basis(basis, D_init: np.ndarray, R: int, xhat: np.ndarray, K: int, n_iter: int, tau: float = TAU):
    """rksvd in the coordinate layout of either basis (see rksvd_update_basis)."""
    D = np.asarray(D_init, dtype=np.float64).copy()
    M = D.shape[0]
    history = []
    for _ in range(n_iter):
        code = omp(augmented_dictionary_basis(basis, D, R), xhat, K, M, tau)
        history.append(float(code.resid2.sum()))
        D, _, _ = rksvd_update_basis(basis, D, R, xhat, code)
    code = omp(augmented_dictionary_basis(basis, D, R), xhat, K, M, tau)
    history.append(float(code.resid2.sum()))
    return D, code, history


def rksvd_update(D_hat: np.ndarray, R: int, S: int, T: int, xhat: np.ndarray, code: Code):
    """Atom update of rotational K-SVD (Fig. 2, the loop over m; Sec. II-C).

    For each atom m, every patch p whose code uses m contributes one column
    S_{-r0} (x_p - D b_p) to Y_m: b_p is the code of p with the entry of atom m at
    angle r0 removed, so the column is what atom m has to explain, turned upright
    with respect to m.  The new atom is the first left singular vector of Y_m.
    Atoms used by no patch are reset (see the module header).

    D_hat [M, B] is the dictionary the codes were computed with; xhat [P, B].
    Returns (D_new [M, B], usage [M], reset [M]) where reset[m] is the patch an
    unused atom was reset to (-1 otherwise).
    """
    return _rksvd_update(D_hat, R, xhat, code, lambda v, th: steer(v, th, S, T))


def _rksvd_update(D_hat: np.ndarray, R: int, xhat: np.ndarray, code: Code, steer_fn):
    """The steps of rksvd_update with the steering S_theta given as steer_fn(v, theta)."""
    D_hat = np.asarray(D_hat, dtype=np.float64)
    xhat = np.asarray(xhat, dtype=np.float64)
    M, B = D_hat.shape
    P, K = code.atom.shape
    D_new = D_hat.copy()
    usage = np.zeros(M, np.int64)
    for m in range(M):
        cols = []
        for p in range(P):
            slots = [i for i in range(K) if code.atom[p, i] == m]
            if not slots:
                continue
            i0 = slots[0]
            r0 = int(code.angle[p, i0])
            others = np.zeros(B)
            for i in range(K):
                if i != i0 and code.atom[p, i] >= 0:
                    theta = 2 * np.pi * code.angle[p, i] / R
                    others += code.coef[p, i] * steer_fn(D_hat[code.atom[p, i]], theta)
            cols.append(steer_fn(xhat[p] - others, -2 * np.pi * r0 / R))
        usage[m] = len(cols)
        if cols:
            Y = np.stack(cols, axis=1)                       # [B, n_m]
            U, _, _ = np.linalg.svd(Y, full_matrices=False)
            D_new[m] = _sign_like(U[:, 0], D_hat[m])
    reset = -np.ones(M, np.int64)
    order = sorted(range(P), key=lambda p: (-float(code.resid2[p]), p))
    nxt = 0
    for m in range(M):
        if usage[m] > 0:
            continue
        if nxt == P or code.resid2[order[nxt]] <= 0:
            break
        p = order[nxt]
        D_new[m] = xhat[p] / np.linalg.norm(xhat[p])
        reset[m] = p
        nxt += 1
    return D_new, usage, reset


def rksvd(D_init: np.ndarray, R: int, S: int, T: int, xhat: np.ndarray, K: int, n_iter: int,
          tau: float = TAU):
    """Rotational K-SVD in hat coordinates (Fig. 2 with R_r -> S_r, Sec. II-E):
    n_iter rounds of pursuit and atom update from D_init, then one more pursuit.
    Returns (D [M, B], codes of the final dictionary, coding error sum_p ||r_p||^2
    after each round's pursuit)."""
    D = np.asarray(D_init, dtype=np.float64).copy()
    M = D.shape[0]
    history = []
    for _ in range(n_iter):
        code = omp(augmented_dictionary(D, R, S, T), xhat, K, M, tau)
        history.append(float(code.resid2.sum()))
        D, _, _ = rksvd_update(D, R, S, T, xhat, code)
    code = omp(augmented_dictionary(D, R, S, T), xhat, K, M, tau)
    history.append(float(code.resid2.sum()))
    return D, code, history


# --------------------------------------------------------------------------- classifier
def classify(D_list, R: int, S: int, T: int, xhat: np.ndarray, K: int, tau: float = TAU):
    """Label of every patch: the class whose dictionary codes it with the smallest
    squared error (Sec. III-B, "Classifier"; readings in the module header).

    D_list: C dictionaries [M_c, B].  Returns (label [P] int, sse [P, C])."""
    sse = []
    for D in D_list:
        D = np.asarray(D, dtype=np.float64)
        code = omp(augmented_dictionary(D, R, S, T), xhat, K, D.shape[0], tau)
        sse.append(code.resid2)
    sse = np.stack(sse, axis=1) if sse else np.zeros((len(xhat), 0))
    label = np.argmin(sse, axis=1) if sse.shape[1] else np.zeros(len(xhat), np.int64)
    return label, sse


def label_histogram(label: np.ndarray, offsets: np.ndarray, C: int) -> np.ndarray:
    """Per group of consecutive patches [offsets[g], offsets[g+1]): the frequencies of
    the C labels (a group without patches has all zeros)."""
    G = len(offsets) - 1
    hist = np.zeros((G, C))
    for g in range(G):
        lab = np.asarray(label[offsets[g]:offsets[g + 1]])
        if lab.size:
            hist[g] = np.bincount(lab, minlength=C)[:C] / lab.size
    return hist


def chi2(a: np.ndarray, b: np.ndarray) -> float:
    """d(a, b) = sum_i (a_i - b_i)^2 / (a_i + b_i) over the bins with a_i + b_i > 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = a + b
    keep = s > 0
    return float(np.sum((a[keep] - b[keep]) ** 2 / s[keep]))


def nearest_chi2(train: np.ndarray, test: np.ndarray):
    """For each test histogram, the training histogram at the smallest chi^2 distance
    (ties: smaller training index).  Returns (index [Q], distance [Q])."""
    idx = np.zeros(len(test), np.int64)
    dist = np.zeros(len(test))
    for q in range(len(test)):
        d = [chi2(test[q], train[j]) for j in range(len(train))]
        idx[q] = int(np.argmin(d))
        dist[q] = d[idx[q]]
    return idx, dist


# --------------------------------------------------------------------------- rotation
def _keys(t: float, a: float = -0.5) -> float:
    """Keys' cubic convolution kernel."""
    t = abs(t)
    if t <= 1.0:
        return (a + 2.0) * t ** 3 - (a + 3.0) * t ** 2 + 1.0
    if t < 2.0:
        return a * t ** 3 - 5.0 * a * t ** 2 + 8.0 * a * t - 4.0 * a
    return 0.0


def rotation_matrix(N: int, theta: float, mode: str) -> np.ndarray:
    """The N^2 x N^2 matrix (row-major pixels) that rotates a patch by theta with
    nearest-neighbour or bicubic interpolation (readings in the module header)."""
    c = (N - 1) / 2.0
    Rm = np.zeros((N * N, N * N))
    cs, sn = np.cos(theta), np.sin(theta)
    for i in range(N):
        for j in range(N):
            x, y = j - c, c - i
            xs, ys = cs * x + sn * y, -sn * x + cs * y        # R_{-theta} (x, y)
            col, row = c + xs, c - ys                          # fractional source pixel
            q = i * N + j
            if mode == "nearest":
                r0, c0 = int(np.floor(row + 0.5)), int(np.floor(col + 0.5))
                if 0 <= r0 < N and 0 <= c0 < N:
                    Rm[q, r0 * N + c0] = 1.0
            elif mode == "bicubic":
                r0, c0 = int(np.floor(row)), int(np.floor(col))
                for di in range(-1, 3):
                    for dj in range(-1, 3):
                        rr, cc = r0 + di, c0 + dj
                        if 0 <= rr < N and 0 <= cc < N:
                            w = _keys(row - rr) * _keys(col - cc)
                            if w != 0.0:
                                Rm[q, rr * N + cc] += w
            else:
                raise ValueError("mode must be 'nearest' or 'bicubic'")
    return Rm


def rotate_interp(patches: np.ndarray, theta: float, mode: str) -> np.ndarray:
    """Patches [P, N, N] rotated by theta (counter-clockwise) by interpolation."""
    P, N, _ = patches.shape
    Rm = rotation_matrix(N, theta, mode)
    return (patches.reshape(P, N * N) @ Rm.T).reshape(P, N, N)


def rotate_steer(basis: Basis, patches: np.ndarray, theta: float) -> np.ndarray:
    """Steering-based rotation Phi S_theta (Phi^T Phi)^{-1} Phi^T x (Sec. III-C), in either basis."""
    return to_pixels(basis, steer_basis(basis, project(basis, patches), theta))


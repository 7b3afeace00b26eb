"""FP64 CPU oracle of the neural multigrid V-cycle (TEST INFRASTRUCTURE ONLY).

This module is the slow, plain reference that the GPU library is checked
against.  Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does, and it shares no code,
header, table or constant generator with the HIP library.

Every array is a CPU ``torch.float64`` tensor.  Batched layouts are
``[B, n]`` (1D) and ``[B, n, n]`` (2D, row-major ``[row][col]``).  Operators
are formed as dense matrices from their definitions; library primitives used
as single steps are matrix products, ``conv1d``/``conv2d`` (PyTorch
cross-correlation) for the CNN smoother, a Cholesky factorisation with two
triangular solves, and autograd for the loss gradient.

What the paper fixes and how each piece is pinned (tests marked ``not gpu``):

* Problem (Sec. 2.1, eq. "integral equation"; 2D Kronecker form Sec. 4.2):
  the regularised system ``(K^T K + alpha I) u = b`` with a truncated Gaussian
  convolution matrix ``K``; 2D uses ``K2 = K (x) K``.  Pinned by brute force
  (dense Toeplitz / Kronecker matrices), symmetry and positive definiteness.
* Operator variants: ``alpha I + K`` (2D ``alpha I (x) I + K (x) K``) as the
  paper writes it, and the 1D anisotropic ``alpha D + K`` (Sec. 4.1).  Pinned
  by dense definitions, the spectrum from the eigenvalues of ``K``, the
  discrete energy identity of ``D`` and its constant-coefficient closed form.
* Grids and transfers (Sec. 2.3, Algorithm 1): linear interpolation ``P`` and
  full weighting ``R = P^T / 2^d``; Galerkin coarse operators
  ``A_{l+1} = R A_l P``.  Pinned by adjointness, exact interpolation of
  linear functions and a dense RAP product.
* Coarse solve (Algorithm 1, coarsest level): Cholesky of the dense coarse
  matrix.  Pinned against a dense LU solve.
* Exact fine-level solve for large grids: eigendecomposition of ``G_1``
  (the Kronecker operator is diagonal in the tensor eigenbasis).  Pinned
  against a dense solve on small grids.
* Neural smoother (Algorithm 2 / Algorithm 4 pre-smoothing step):
  ``h = ||b|| N(b / ||b||)`` with a bias-free ReLU CNN.  Pinned by an explicit
  dense convolution matrix and positive homogeneity.
* Filter ``F'_l`` (Sec. 3.2, Algorithm 3; 2D Sec. 3.3, Algorithm 4): ramp mask
  in an orthonormal DCT-II basis on the level grid.  Pinned by orthogonality
  and the closed-form response on single basis vectors.
* FNO smoother (Sec. 3.1 neural operators; appendix network description):
  lift, Fourier layers (truncated real DFT, complex mode mixing, "same"
  convolution, bias, GELU), projection.  Pinned by an explicit DFT-matrix
  evaluation of the spectral layer, a dense convolution matrix, the
  closed-form response of a single retained mode, and the erf definition
  of GELU.
* Cycle (Algorithms 1, 2, 4): pinned by the residual-driven identity, the
  cycle decomposition identity of Sec. 3.2, the exact-smoother and one-level
  cases, and reduction to a textbook damped-Jacobi V-cycle.
* Solve (outer iteration, Sec. 2.3): pinned by a dense direct solve.
* Level-wise loss (Sec. 3.2 eq. "loss_2_modified", 2D eq. "loss_3"): pinned
  by the Parseval identity of Sec. 3.2 and central finite differences of the
  gradient.
* Combined loss (Sec. 3.2 eq. "loss_1"): pinned by the two-grid error
  propagation identity built from dense matrices and by central finite
  differences of the joint gradient over all levels.
* Level-wise loss value: pinned by rebuilding every level's unresolved error
  from the recorded cycle with direct hat-function interpolation to the
  finest grid and measuring its band energy in the eigenbasis of the
  Neumann second-difference matrix (the DCT-II basis found another way).
* FNO smoother wrapper ``||b|| N(b/||b||)``: pinned by a pure-Python
  evaluation of the whole FNO on a small 1D grid with the norm summed by
  hand, its degree-one homogeneity (the network itself has biases, so only
  the wrapper makes it homogeneous) and ``h = 0`` at ``b = 0``.
* Training data (Algorithm 5 DataGeneration): pinned by a dense textbook
  damped-Jacobi cycle (the rollout is then linear, ``e <- E e``), by one
  rollout with the exact finest-level smoother (the error vanishes), and by
  ``y = A e`` against the dense operator.

Parity unpinned: iteration counts of trained or seeded neural cycles (the
paper prints no worked values for them); they are compared GPU-vs-oracle only.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import torch
import torch.nn.functional as F

DT = torch.float64

# ---------------------------------------------------------------------------
# Problem: grid, kernel, operator (Sec. 2.1; Sec. 4.1 / 4.2 experiments)
# ---------------------------------------------------------------------------


def mesh_width(n: int) -> float:
    """Mesh size of a grid with ``n`` interior points and zero boundary values.

    Sec. 2.1 partitions [0,1] into equal cells; the unknowns are the ``n``
    interior nodes, so there are ``n + 1`` cells and ``h = 1/(n+1)``.
    """
    return 1.0 / (n + 1)


def gaussian_radius(n: int, s: float, trunc: float = 4.0) -> int:
    """Truncation radius in grid points: every tap with ``|j| h <= trunc*s``."""
    h = mesh_width(n)
    return int(math.floor(trunc * s / h + 1e-9))


def gaussian_taps(n: int, s: float, trunc: float = 4.0) -> torch.Tensor:
    """Quadrature weights ``k_j = h g(j h)`` of the Gaussian kernel, j=-R..R.

    ``g(z) = exp(-z^2/(2 s^2)) / (sqrt(2 pi) s)`` is the smooth convolution
    kernel of Sec. 2.1 (Gaussian smoothing kernel of Sec. 4.1), discretised by
    the rectangle rule on the uniform mesh; no renormalisation after
    truncation.
    """
    h = mesh_width(n)
    R = gaussian_radius(n, s, trunc)
    j = torch.arange(-R, R + 1, dtype=DT)
    return h * torch.exp(-(j * h) ** 2 / (2.0 * s * s)) / (math.sqrt(2.0 * math.pi) * s)


def conv_matrix(n: int, s: float, trunc: float = 4.0) -> torch.Tensor:
    """Dense Toeplitz convolution matrix ``K[i, j] = h g(x_i - x_j)`` (Sec. 2.1).

    Entries with ``|x_i - x_j| > trunc*s`` are zero; zero boundary values mean
    the matrix is the ``n x n`` section of the infinite Toeplitz operator.
    """
    taps = gaussian_taps(n, s, trunc)
    R = (taps.numel() - 1) // 2
    K = torch.zeros(n, n, dtype=DT)
    for i in range(n):
        for j in range(max(0, i - R), min(n, i + R + 1)):
            K[i, j] = taps[j - i + R]
    return K


def anisotropic_regulariser(n: int, a: Optional[Callable[[float], float]] = None) -> torch.Tensor:
    """Tridiagonal ``D`` of the 1D regulariser ``-(a u')'`` (Sec. 4.1,
    anisotropic case, ``a(z) = 1 + 0.5 sin(2 pi z)``), zero boundary values.

    Conservative three-point differences with ``a`` taken at the cell
    midpoints ``(i + 1/2) h``: ``(D v)_i = a_{i-1/2} (v_i - v_{i-1}) -
    a_{i+1/2} (v_{i+1} - v_i)``.  The factor ``1/h^2`` is left out (reading:
    the paper's alphas for this case match those of the ``alpha I`` case, so
    ``D`` carries the same O(1) scale as ``I``).
    """
    if a is None:
        a = lambda z: 1.0 + 0.5 * math.sin(2.0 * math.pi * z)
    h = mesh_width(n)
    D = torch.zeros(n, n, dtype=DT)
    for i in range(n):
        left, right = a((i + 0.5) * h), a((i + 1.5) * h)
        D[i, i] = left + right
        if i > 0:
            D[i, i - 1] = -left
        if i + 1 < n:
            D[i, i + 1] = -right
    return D


# ---------------------------------------------------------------------------
# Grid hierarchy and transfers (Sec. 2.3, Algorithm 1)
# ---------------------------------------------------------------------------


def prolongation_matrix(nc: int) -> torch.Tensor:
    """Linear interpolation from ``nc`` coarse to ``2 nc + 1`` fine points.

    Coarse node i sits on fine node 2i+1; fine nodes 2i and 2i+2 take half of
    it; the zero boundary supplies the missing neighbours (Sec. 2.3: the
    interpolation matrix between consecutive grids of mesh h and 2h).
    """
    nf = 2 * nc + 1
    P = torch.zeros(nf, nc, dtype=DT)
    for i in range(nc):
        P[2 * i + 1, i] = 1.0
        P[2 * i, i] += 0.5
        P[2 * i + 2, i] += 0.5
    return P


def restriction_matrix(nc: int) -> torch.Tensor:
    """Full weighting in 1D: ``R = P^T / 2`` (weights 1/4, 1/2, 1/4)."""
    return prolongation_matrix(nc).T / 2.0


@dataclass
class Level:
    """One grid level: ``A_l = alpha M_l (x) M_l + G_l (x) G_l`` (2D).

    In 1D the same level is ``A_l = alpha M_l + G_l``.  ``M_1 = I`` and
    ``G_1 = K^T K``; coarser factors come from the Galerkin product of
    Algorithm 1 applied to each Kronecker factor separately, which is exact
    because ``R (B (x) B) P = (R1 B P1) (x) (R1 B P1)``.
    """

    n: int
    M: torch.Tensor
    G: torch.Tensor
    P: Optional[torch.Tensor] = None  # interpolation from the next coarser level


@dataclass
class Hierarchy:
    dim: int
    n: int
    s: float
    levels: List[Level] = field(default_factory=list)

    @property
    def L(self) -> int:
        return len(self.levels)


def build_hierarchy(n: int, s: float, levels: int, dim: int = 2, trunc: float = 4.0,
                    form: str = "normal") -> Hierarchy:
    """Hierarchy of Algorithm 1: ``n_{l+1} = (n_l - 1)/2`` and Galerkin RAP.

    ``form`` picks the fine operator: ``"normal"`` is ``alpha I + K^T K`` (2D:
    ``alpha I + (K (x) K)^T (K (x) K)``), ``"kernel"`` is the paper's own
    ``alpha I + K`` (Sec. 2.1; 2D ``alpha I (x) I + K (x) K`` of Sec. 4.2) and
    ``"aniso"`` is ``alpha D + K`` with the anisotropic regulariser (1D only,
    Sec. 4.1).
    """
    if dim not in (1, 2):
        raise ValueError("dim must be 1 or 2")
    if form not in ("normal", "kernel", "aniso"):
        raise ValueError("form must be 'normal', 'kernel' or 'aniso'")
    if form == "aniso" and dim != 1:
        raise ValueError("the anisotropic regulariser is one-dimensional")
    K = conv_matrix(n, s, trunc)
    G = K.T @ K if form == "normal" else K
    M = anisotropic_regulariser(n) if form == "aniso" else torch.eye(n, dtype=DT)
    H = Hierarchy(dim=dim, n=n, s=s)
    H.levels.append(Level(n=n, M=M, G=G))
    for _ in range(1, levels):
        nf = H.levels[-1].n
        if nf < 3 or nf % 2 == 0:
            raise ValueError("grid cannot be coarsened further")
        nc = (nf - 1) // 2
        P = prolongation_matrix(nc)
        R = P.T / 2.0
        M = R @ M @ P
        G = R @ G @ P
        H.levels[-1].P = P
        H.levels.append(Level(n=nc, M=M, G=G))
    return H


def apply_operator(H: Hierarchy, l: int, x: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """``A_l x`` per right-hand side; ``alpha`` has shape ``[B]``."""
    lv = H.levels[l]
    if H.dim == 1:
        return alpha[:, None] * (x @ lv.M.T) + x @ lv.G.T
    return alpha[:, None, None] * (lv.M @ x @ lv.M.T) + lv.G @ x @ lv.G.T


def dense_operator(H: Hierarchy, l: int, alpha: float) -> torch.Tensor:
    """Dense matrix of ``A_l`` acting on the row-major vectorisation."""
    lv = H.levels[l]
    if H.dim == 1:
        return alpha * lv.M + lv.G
    return alpha * torch.kron(lv.M, lv.M) + torch.kron(lv.G, lv.G)


def restrict(H: Hierarchy, l: int, r: torch.Tensor) -> torch.Tensor:
    """``I_l^{l+1} r``: full weighting from level ``l`` to ``l+1``."""
    P = H.levels[l].P
    R = P.T / 2.0
    if H.dim == 1:
        return r @ R.T
    return R @ r @ R.T


def prolong(H: Hierarchy, l: int, e: torch.Tensor) -> torch.Tensor:
    """``I_{l+1}^l e``: linear (2D: bilinear) interpolation to level ``l``."""
    P = H.levels[l].P
    if H.dim == 1:
        return e @ P.T
    return P @ e @ P.T


def prolong_to_finest(H: Hierarchy, l: int, e: torch.Tensor) -> torch.Tensor:
    """``I_l^1 e = I_2^1 ... I_l^{l-1} e``."""
    for k in range(l - 1, -1, -1):
        e = prolong(H, k, e)
    return e


def transfer_index_maps(nc: int):
    """Integer index maps of the 1D transfers, by enumerating nonzeros of ``P``.

    Returns ``(restrict_map, prolong_map)``.  ``restrict_map[i]`` lists the fine
    indices read by coarse node ``i`` (ascending) with their weights;
    ``prolong_map[p]`` lists the coarse indices read by fine node ``p``.
    """
    P = prolongation_matrix(nc)
    R = P.T / 2.0
    rmap = [[(int(j), float(R[i, j])) for j in torch.nonzero(R[i]).flatten()] for i in range(nc)]
    pmap = [[(int(j), float(P[p, j])) for j in torch.nonzero(P[p]).flatten()] for p in range(P.shape[0])]
    return rmap, pmap


# ---------------------------------------------------------------------------
# Coarsest-grid direct solve (Algorithm 1: exact solve at l = L)
# ---------------------------------------------------------------------------


def coarse_factor(H: Hierarchy, alpha: float) -> torch.Tensor:
    """Lower Cholesky factor of the dense coarsest-level matrix."""
    A = dense_operator(H, H.L - 1, alpha)
    return torch.linalg.cholesky(A)


def coarse_solve(H: Hierarchy, y: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """``x_L = (A_L)^{-1} y_L`` by Cholesky and two triangular solves."""
    out = torch.empty_like(y)
    for b in range(y.shape[0]):
        Lf = coarse_factor(H, float(alpha[b]))
        v = y[b].reshape(-1, 1)
        z = torch.linalg.solve_triangular(Lf, v, upper=False)
        w = torch.linalg.solve_triangular(Lf.T, z, upper=True)
        out[b] = w.reshape(y[b].shape)
    return out


def direct_solve(H: Hierarchy, y: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    """Exact solution of the finest system ``A_1 x = y`` when ``M_1 = I``.

    ``A_1 = alpha I + G (x) G`` (2D) is diagonalised by ``Q (x) Q`` with
    ``G = Q diag(lam) Q^T``: ``x = Q [(Q^T Y Q) / (alpha + lam_i lam_j)] Q^T``;
    in 1D ``x = Q diag(1 / (alpha + lam)) Q^T y``.  One symmetric
    eigendecomposition of ``n x n`` serves every right-hand side, so this
    reaches grids far beyond a dense factorisation of ``A_1``.
    """
    lv = H.levels[0]
    if not torch.equal(lv.M, torch.eye(lv.n, dtype=DT)):
        raise ValueError("direct_solve needs M_1 = I")
    lam, Q = torch.linalg.eigh(lv.G)
    out = torch.empty_like(y)
    for b in range(y.shape[0]):
        a = float(alpha[b])
        if H.dim == 1:
            out[b] = Q @ ((Q.T @ y[b]) / (a + lam))
        else:
            out[b] = Q @ ((Q.T @ y[b] @ Q) / (a + lam[:, None] * lam[None, :])) @ Q.T
    return out


# ---------------------------------------------------------------------------
# Smoothers (Sec. 2.2 weighted Jacobi; Algorithms 2-4 neural smoother)
# ---------------------------------------------------------------------------


def cnn_forward(weights: Sequence[torch.Tensor], x: torch.Tensor, dim: int) -> torch.Tensor:
    """Bias-free CNN: conv, ReLU, ..., conv (no activation after the last).

    ``weights[i]`` has shape ``[Cout, Cin, k]`` (1D) or ``[Cout, Cin, k, k]``
    (2D); cross-correlation with zero "same" padding.
    """
    z = x.unsqueeze(1)
    conv = F.conv1d if dim == 1 else F.conv2d
    for i, w in enumerate(weights):
        z = conv(z, w, padding=w.shape[-1] // 2)
        if i + 1 < len(weights):
            z = torch.relu(z)
    return z.squeeze(1)


def fno_modes(n: int, k: int) -> int:
    """Retained Fourier modes per axis on an ``n``-point grid: ``min(k, n // 2)``
    (in 2D the two retained row blocks ``[0, k)`` and ``[n - k, n)`` stay
    disjoint)."""
    return min(k, n // 2)


def gelu(x: torch.Tensor) -> torch.Tensor:
    """GELU with the exact error function, ``x Phi(x)``."""
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def spectral_conv(z: torch.Tensor, R: torch.Tensor, k: int, dim: int) -> torch.Tensor:
    """``DFT^-1 (R . DFT(z))`` keeping the ``k`` lowest modes per axis (the
    Fourier layer of the appendix's network description).

    ``z``: ``[B, C, n]`` or ``[B, C, n, n]`` real; the DFT is the real FFT over
    the grid values.  1D: ``R`` is complex ``[C, C, k]`` and mode ``m < k``
    maps as ``out[co, m] = sum_ci in[ci, m] R[ci, co, m]``.  2D: ``R`` is
    complex ``[2, C, C, k, k]`` for the row blocks ``[0, k)`` and
    ``[n - k, n)`` times columns ``[0, k)`` of the half spectrum.  All other
    modes are zero."""
    n = z.shape[-1]
    if dim == 1:
        zf = torch.fft.rfft(z, dim=-1)
        out = torch.zeros_like(zf)
        out[..., :k] = torch.einsum("bim,iom->bom", zf[..., :k], R)
        return torch.fft.irfft(out, n=n, dim=-1)
    zf = torch.fft.rfft2(z, dim=(-2, -1))
    out = torch.zeros_like(zf)
    out[..., :k, :k] = torch.einsum("bixy,ioxy->boxy", zf[..., :k, :k], R[0])
    out[..., n - k:, :k] = torch.einsum("bixy,ioxy->boxy", zf[..., n - k:, :k], R[1])
    return torch.fft.irfft2(out, s=(n, n), dim=(-2, -1))


def fno_forward(params: dict, x: torch.Tensor, dim: int, modes: int) -> torch.Tensor:
    """Fourier neural operator of the appendix: a pointwise fully connected
    lift ``1 -> C`` (weight and bias), Fourier layers
    ``z <- sigma(DFT^-1 R DFT z + W z + B)`` with ``W`` a "same"-padded
    convolution and ``sigma`` = GELU, then a pointwise projection ``C -> 1``.

    ``params``: ``lift_w [C]``, ``lift_b [C]``, ``layers`` = list of dicts
    with ``R`` (complex, see :func:`spectral_conv`), ``W [C, C, ks(, ks)]``,
    ``B [C]``; ``proj_w [C]``, ``proj_b`` (scalar tensor)."""
    n = x.shape[-1]
    k = fno_modes(n, modes)
    shape = (1, -1) + (1,) * dim
    z = params["lift_w"].reshape(shape) * x.unsqueeze(1) + params["lift_b"].reshape(shape)
    conv = F.conv1d if dim == 1 else F.conv2d
    for layer in params["layers"]:
        R = layer["R"][..., :k] if dim == 1 else layer["R"][..., :k, :k]
        s = spectral_conv(z, R, k, dim)
        w = conv(z, layer["W"], bias=layer["B"], padding=layer["W"].shape[-1] // 2)
        z = gelu(s + w)
    return (params["proj_w"].reshape(shape) * z).sum(dim=1) + params["proj_b"]


def fno_smoother(params: dict, dim: int, modes: int) -> Callable:
    """``h = ||b|| N(b / ||b||)`` with the FNO as ``N``; zero for ``b = 0``."""

    def apply(H, l, b, alpha):
        nrm = batch_norm2(b)
        safe = torch.where(nrm > 0, nrm, torch.ones_like(nrm))
        shape = (-1,) + (1,) * (b.dim() - 1)
        out = fno_forward(params, b / safe.reshape(shape), dim, modes) * nrm.reshape(shape)
        return torch.where(nrm.reshape(shape) > 0, out, torch.zeros_like(out))

    return apply


def batch_norm2(b: torch.Tensor) -> torch.Tensor:
    """Per-sample Euclidean norm (2D: Frobenius norm = 2-norm of Vec)."""
    return torch.sqrt((b * b).reshape(b.shape[0], -1).sum(dim=1))


def neural_smoother(weights: Sequence[torch.Tensor], dim: int) -> Callable:
    """``h = N(b/||b||) ||b||`` (Algorithm 2 pre-smoothing; Algorithm 4 in 2D).

    A zero residual gives a zero correction.
    """

    def apply(H, l, b, alpha):
        nrm = batch_norm2(b)
        safe = torch.where(nrm > 0, nrm, torch.ones_like(nrm))
        shape = (-1,) + (1,) * (b.dim() - 1)
        out = cnn_forward(weights, b / safe.reshape(shape), dim) * nrm.reshape(shape)
        return out

    return apply


def jacobi_diagonal(H: Hierarchy, l: int, alpha: torch.Tensor) -> torch.Tensor:
    """Diagonal of ``A_l`` per right-hand side, shaped like one sample batch."""
    lv = H.levels[l]
    m = torch.diagonal(lv.M)
    g = torch.diagonal(lv.G)
    if H.dim == 1:
        return alpha[:, None] * m[None, :] + g[None, :]
    return alpha[:, None, None] * (m[:, None] * m[None, :])[None] + (g[:, None] * g[None, :])[None]


def jacobi_smoother(omegas: Sequence[float]) -> Callable:
    """Weighted Jacobi ``h = omega_l D_l^{-1} b`` (Sec. 2.2)."""

    def apply(H, l, b, alpha):
        return omegas[l] * b / jacobi_diagonal(H, l, alpha)

    return apply


# ---------------------------------------------------------------------------
# Frequency masks and the filter F'_l (Sec. 2.3 bands; Sec. 3.2 / 3.3 masks)
# ---------------------------------------------------------------------------


def dct2_matrix(n: int) -> torch.Tensor:
    """Orthonormal DCT-II: ``C[k, i] = c_k cos(pi k (2i+1) / (2n))``.

    Row ``k`` carries the frequency ``omega_k = pi k / n`` in ``[0, pi)``.
    """
    k = torch.arange(n, dtype=DT)[:, None]
    i = torch.arange(n, dtype=DT)[None, :]
    C = torch.cos(math.pi * k * (2.0 * i + 1.0) / (2.0 * n)) * math.sqrt(2.0 / n)
    C[0] *= 1.0 / math.sqrt(2.0)
    return C


def max_frequency_index(n: int, dim: int) -> torch.Tensor:
    k = torch.arange(n, dtype=torch.int64)
    if dim == 1:
        return k
    return torch.maximum(k[:, None], k[None, :])


def loss_mask(N: int, l: int, kind: str, dim: int) -> torch.Tensor:
    """Mask ``m_l`` (1D) / ``M_l`` (2D) on the finest grid for level ``l >= 1``.

    Frequencies are ``omega = pi k / N`` per axis and the 2D band variable is
    ``max(|omega_1|, |omega_2|)`` (Sec. 2.3, 2D band decomposition).

    ``kind="ramp"``: the paper's mask ``sqrt(omega / (pi / 2^(l-1)))`` for
    ``omega <= pi / 2^(l-1)`` and zero above (Sec. 3.2, 2D in Sec. 3.3).
    ``kind="band"``: indicator of the level's own high band
    ``pi/2^l < omega <= pi/2^(l-1)`` (the band Phi_l of Sec. 2.3).
    Band membership is decided in integers so both sides agree exactly.
    """
    k = max_frequency_index(N, dim)
    p = 2 ** (l - 1)
    visible = k * p <= N
    if kind == "ramp":
        val = torch.sqrt(k.to(DT) * p / N)
        return torch.where(visible, val, torch.zeros_like(val))
    if kind == "band":
        return ((k * 2 * p > N) & visible).to(DT)
    raise ValueError(kind)


def fprime_mask(n: int, dim: int) -> torch.Tensor:
    """``m'_l`` / ``M'_l``: the ramp over the whole range visible on a grid of
    ``n`` points, i.e. ``sqrt(omega / pi)`` with ``omega = pi k / n``."""
    k = max_frequency_index(n, dim)
    return torch.sqrt(k.to(DT) / n)


def dct_forward(x: torch.Tensor, C: torch.Tensor, dim: int) -> torch.Tensor:
    if dim == 1:
        return x @ C.T
    return C @ x @ C.T


def dct_inverse(X: torch.Tensor, C: torch.Tensor, dim: int) -> torch.Tensor:
    if dim == 1:
        return X @ C
    return C.T @ X @ C


def fprime(h: torch.Tensor, dim: int) -> torch.Tensor:
    """``F'_l(h) = C^T (m'_l * (C h))`` on the level grid (Algorithms 3, 4)."""
    n = h.shape[-1]
    C = dct2_matrix(n)
    return dct_inverse(fprime_mask(n, dim) * dct_forward(h, C, dim), C, dim)


# ---------------------------------------------------------------------------
# The cycle (Algorithm 1 skeleton; Algorithms 2-4 with neural smoothers)
# ---------------------------------------------------------------------------


def vcycle(H: Hierarchy, smoothers: Sequence[Callable], x: torch.Tensor, y: torch.Tensor,
           alpha: torch.Tensor, nu1: int = 1, nu2: int = 1, use_fprime: bool = False,
           level: int = 0, record: Optional[list] = None) -> torch.Tensor:
    """One V(nu1, nu2) cycle on level ``level`` (0-based) with initial guess ``x``.

    Coarsest level: exact solve.  Otherwise ``nu1`` smoothing steps
    ``b = y - A x; x += F'(S(b))``, restriction of the residual, recursive
    cycle from zero, interpolation and correction, then ``nu2`` smoothing
    steps with the same smoother.  ``record`` (if given) receives
    ``(level, b, h)`` for every pre-smoothing step.
    """
    if level == H.L - 1:
        return coarse_solve(H, y, alpha)
    S = smoothers[level]
    for _ in range(nu1):
        b = y - apply_operator(H, level, x, alpha)
        h = S(H, level, b, alpha)
        if record is not None:
            record.append((level, b, h))
        x = x + (fprime(h, H.dim) if use_fprime else h)
    r = y - apply_operator(H, level, x, alpha)
    yc = restrict(H, level, r)
    ec = vcycle(H, smoothers, torch.zeros_like(yc), yc, alpha, nu1, nu2, use_fprime, level + 1, record)
    x = x + prolong(H, level, ec)
    for _ in range(nu2):
        b = y - apply_operator(H, level, x, alpha)
        h = S(H, level, b, alpha)
        x = x + (fprime(h, H.dim) if use_fprime else h)
    return x


@dataclass
class SolveResult:
    x: torch.Tensor
    cycles: torch.Tensor           # [B] cycles used per right-hand side
    history: List[torch.Tensor]    # relative residual per right-hand side, before each cycle
    converged: torch.Tensor        # [B] bool


def relative_residual(H: Hierarchy, x: torch.Tensor, y: torch.Tensor, alpha: torch.Tensor) -> torch.Tensor:
    r = y - apply_operator(H, 0, x, alpha)
    return batch_norm2(r) / batch_norm2(y)


def solve(H: Hierarchy, smoothers: Sequence[Callable], y: torch.Tensor, alpha: torch.Tensor,
          tol: float = 1e-6, max_cycles: int = 100, nu1: int = 1, nu2: int = 1,
          use_fprime: bool = False) -> SolveResult:
    """Outer iteration ``x^{t+1} = MG(A, x^t, y)`` from ``x^0 = 0`` (Sec. 2.3).

    Each right-hand side stops independently once its relative residual is at
    most ``tol``; a stopped right-hand side is left unchanged.
    """
    x = torch.zeros_like(y)
    cycles = torch.zeros(y.shape[0], dtype=torch.int64)
    active = torch.ones(y.shape[0], dtype=torch.bool)
    history = []
    for _ in range(max_cycles + 1):
        rel = relative_residual(H, x, y, alpha)
        history.append(rel.clone())
        active = active & (rel > tol) & torch.isfinite(rel)
        if not bool(active.any()) or len(history) > max_cycles:
            break
        xn = vcycle(H, smoothers, x, y, alpha, nu1, nu2, use_fprime)
        shape = (-1,) + (1,) * (y.dim() - 1)
        x = torch.where(active.reshape(shape), xn, x)
        cycles += active.to(torch.int64)
    rel = relative_residual(H, x, y, alpha)
    return SolveResult(x=x, cycles=cycles, history=history, converged=rel <= tol)


# ---------------------------------------------------------------------------
# Level-wise training loss and its gradient (Sec. 3.2 eq. loss_2_modified,
# 2D eq. loss_3; Algorithm 5 training step)
# ---------------------------------------------------------------------------


def level_losses(H: Hierarchy, weights: Sequence[Sequence[torch.Tensor]], e: torch.Tensor,
                 alpha: torch.Tensor, mask_kind: str = "ramp", use_fprime: bool = False,
                 make_smoother: Optional[Callable] = None):
    """Per-level losses ``L_l`` for a batch of true solutions ``e`` (``y = A e``).

    The cycle runs once from zero with pre-smoothing only.  For level ``l``
    (1-based) the unresolved error on the finest grid is
    ``e - sum_{k<l} I_k^1 F'_k(h_k) - I_l^1 h_l`` and ``L_l`` is the mean over
    samples of the squared masked DCT-II coefficients of it.  The returned
    losses are built so that ``sum(L).backward()`` leaves ``dL_l/dtheta_l`` in
    ``weights[l]`` only: corrections of earlier levels enter as constants.
    """
    N = H.n
    Nb = e.shape[0]
    C = dct2_matrix(N)
    y = apply_operator(H, 0, e, alpha)
    yl = y
    resolved = torch.zeros_like(e)
    losses = []
    for l in range(H.L - 1):
        b = yl.detach()  # x* = 0 at every level of a cycle started from zero
        sm = make_smoother(weights[l]) if make_smoother else neural_smoother(weights[l], H.dim)
        h = sm(H, l, b, alpha)
        err = e - resolved - prolong_to_finest(H, l, h)
        m = loss_mask(N, l + 1, mask_kind, H.dim)
        losses.append(((m * dct_forward(err, C, H.dim)) ** 2).sum() / Nb)
        with torch.no_grad():
            hc = fprime(h.detach(), H.dim) if use_fprime else h.detach()
            resolved = resolved + prolong_to_finest(H, l, hc)
            yl = restrict(H, l, b - apply_operator(H, l, hc, alpha))
    return losses


def level_loss_grads(H: Hierarchy, weights: Sequence[Sequence[torch.Tensor]], e: torch.Tensor,
                     alpha: torch.Tensor, mask_kind: str = "ramp", use_fprime: bool = False):
    """``(losses, grads)`` with ``grads[l][i] = dL_l / d weights[l][i]``."""
    ws = [[w.detach().clone().requires_grad_(True) for w in lw] for lw in weights]
    losses = level_losses(H, ws, e, alpha, mask_kind, use_fprime)
    total = sum(losses)
    total.backward()
    grads = [[w.grad.detach().clone() for w in lw] for lw in ws]
    return torch.stack([x.detach() for x in losses]), grads


def data_generation(H: Hierarchy, smoothers: Sequence[Callable], e: torch.Tensor, alpha: torch.Tensor,
                    k: Sequence[int], nu1: int = 1, nu2: int = 0, use_fprime: bool = False):
    """Training pairs of the DataGeneration procedure of Algorithm 5.

    Sample ``i`` starts from the drawn error ``e_i`` and goes through
    ``k[i]`` rollout cycles with the current smoothers (Algorithm 5 draws
    ``k[i]`` uniformly from ``1..K``; the caller draws it and passes it in):
    ``e_i <- e_i - MG(0, A e_i)``, after which the right-hand side is
    ``y_i = A e_i`` again.  Reading of the printed update ``y <- y - A x``:
    the pair is kept consistent, ``y = A x`` (taken literally it would turn
    ``y`` into ``A MG(0, y)``, which no longer matches ``x``).  The cycle is
    the one the smoothers are trained in, V(nu1, nu2) with or without
    ``F'``.  No gradient flows through the rollout.  Returns ``(e, y)``."""
    out = e.detach().clone()
    with torch.no_grad():
        for i in range(out.shape[0]):
            ei = out[i:i + 1]
            ai = alpha[i:i + 1]
            for _ in range(int(k[i])):
                yi = apply_operator(H, 0, ei, ai)
                ei = ei - vcycle(H, smoothers, torch.zeros_like(ei), yi, ai, nu1, nu2, use_fprime)
            out[i] = ei[0]
        return out, apply_operator(H, 0, out, alpha)


def fno_from_real(p: dict) -> dict:
    """FNO parameters with the spectral weights as real and imaginary parts
    (``R_re``, ``R_im``, as the library stores them) turned into the complex
    ``R`` of :func:`fno_forward`; autograd flows to the real parts."""
    return {"lift_w": p["lift_w"], "lift_b": p["lift_b"], "proj_w": p["proj_w"], "proj_b": p["proj_b"],
            "layers": [{"R": torch.complex(L["R_re"], L["R_im"]), "W": L["W"], "B": L["B"]} for L in p["layers"]]}


def fno_level_loss_grads(H: Hierarchy, params: Sequence[dict], e: torch.Tensor, alpha: torch.Tensor, modes: int,
                         mask_kind: str = "ramp", use_fprime: bool = False):
    """Level-wise losses with FNO smoothers and ``dL_l/dtheta_l`` for every
    real parameter tensor of level ``l`` (same keys as ``params[l]``)."""
    leaves = []

    def leaf(t):
        t = t.detach().clone().requires_grad_(True)
        leaves.append(t)
        return t

    ps = [{"lift_w": leaf(p["lift_w"]), "lift_b": leaf(p["lift_b"]), "proj_w": leaf(p["proj_w"]),
           "proj_b": leaf(p["proj_b"]),
           "layers": [{k: leaf(L[k]) for k in ("R_re", "R_im", "W", "B")} for L in p["layers"]]} for p in params]
    losses = level_losses(H, ps, e, alpha, mask_kind, use_fprime,
                          make_smoother=lambda p: fno_smoother(fno_from_real(p), H.dim, modes))
    sum(losses).backward()
    grads = [{"lift_w": p["lift_w"].grad, "lift_b": p["lift_b"].grad, "proj_w": p["proj_w"].grad,
              "proj_b": p["proj_b"].grad,
              "layers": [{k: L[k].grad for k in ("R_re", "R_im", "W", "B")} for L in p["layers"]]} for p in ps]
    return torch.stack([x.detach() for x in losses]), grads


def cycle_loss(H: Hierarchy, weights: Sequence[Sequence[torch.Tensor]], e: torch.Tensor, alpha: torch.Tensor,
               use_fprime: bool = False) -> torch.Tensor:
    """Combined loss of Sec. 3.2 eq. loss_1: the mean over samples of
    ``||e - NMG(0, A e)||^2`` for one cycle from zero with pre-smoothing only
    (the cycle of Algorithms 2 and 4), the exact coarsest solve included.
    Every level's weights receive gradient, through the residuals that the
    corrections of finer levels leave for coarser ones."""
    S = [neural_smoother(w, H.dim) for w in weights]
    y = apply_operator(H, 0, e, alpha)
    x = vcycle(H, S, torch.zeros_like(e), y, alpha, nu1=1, nu2=0, use_fprime=use_fprime)
    return ((e - x) ** 2).sum() / e.shape[0]


def cycle_loss_grads(H: Hierarchy, weights: Sequence[Sequence[torch.Tensor]], e: torch.Tensor,
                     alpha: torch.Tensor, use_fprime: bool = False):
    """``(loss, grads)`` of eq. loss_1 with ``grads[l][i] = dL / d weights[l][i]``."""
    ws = [[w.detach().clone().requires_grad_(True) for w in lw] for lw in weights]
    loss = cycle_loss(H, ws, e, alpha, use_fprime)
    loss.backward()
    return loss.detach(), [[w.grad.detach().clone() for w in lw] for lw in ws]


def adam_update(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
                lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One bias-corrected Adam step (the optimiser named in Sec. 3.4)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return param - lr * mh / (torch.sqrt(vh) + eps), m, v

"""Seeded synthetic inputs for the DPP sampler: marginal kernels and uniform streams.

This module only builds inputs. It holds none of the sampler's arithmetic and is
shared by the tests, the smoke check and the benchmark (both the GPU path and the
CPU oracle receive exactly the bytes it produces).

Kernels follow the admissibility facts the paper relies on: a Hermitian matrix
is a marginal kernel iff its eigenvalues lie in [0, 1] (Macchi, Sec. 1), a
diagonal similarity of a kernel defines the same DPP (Prop. 2), and an
orthogonal projection of rank k gives samples of size exactly k (Sec. 1).

Random numbers come from numpy's PCG64 (``default_rng(seed)``).
"""
from __future__ import annotations

import numpy as np


def uniform_stream(n: int, seed: int) -> np.ndarray:
    """u_j ~ U[0, 1), FP64, one per index."""
    return np.random.default_rng(seed).random(n)


def greedy_stream(n: int) -> np.ndarray:
    """u_j = 1/2 for every index. With the keep-iff-u_j-below-d_j rule each
    index then takes its likelier outcome given the earlier decisions: the
    greedy maximum-likelihood mode (Sec. 2, after Thm. 2); an exact tie
    d_j = 1/2 excludes j."""
    return np.full(n, 0.5)


def symmetrize_lower(K: np.ndarray) -> np.ndarray:
    """Copy the lower triangle onto the upper one, so K is exactly symmetric."""
    return np.tril(K) + np.tril(K, -1).T


def _orthonormal(rng, rows: int, cols: int) -> np.ndarray:
    """Q factor of the Householder QR of a seeded N(0,1) rows x cols matrix."""
    G = rng.standard_normal((rows, cols))
    Q, _ = np.linalg.qr(G, mode="reduced")
    return Q


def hermitian_kernel(n: int, seed: int, device=None):
    """K = Q diag(lam) Q^T with Q from QR of N(0,1) n x n and lam_i ~ U(0,1).

    With ``device`` (a torch CUDA device) the QR and the product run there in
    FP64 from the same host draws, and a column-major device tensor is
    returned (the same construction; the bytes differ from the host path's)."""
    rng = np.random.default_rng(seed)
    if device is None:
        Q = _orthonormal(rng, n, n)
        lam = rng.random(n)
        return np.asfortranarray(symmetrize_lower((Q * lam) @ Q.T))
    import torch
    G = rng.standard_normal((n, n))
    lam = rng.random(n)
    Q, _ = torch.linalg.qr(torch.from_numpy(G).to(device), mode="reduced")
    K = (Q * torch.from_numpy(lam).to(device)) @ Q.T
    del Q
    K = torch.tril(K) + torch.tril(K, -1).T
    return K.T.contiguous().T


def projection_kernel(n: int, rank: int, seed: int, device=None):
    """K = Q_r Q_r^T with Q_r the Q factor of QR of a seeded N(0,1) n x rank matrix.

    With ``device`` (a torch CUDA device) the QR and the product run on that
    device (FP64) and a device tensor is returned (column-major storage, i.e.
    the transpose view of a row-major buffer; K is symmetric so the bytes are
    the same). The Gaussian matrix is always drawn on the host from the seed.
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, rank))
    if device is None:
        Q, _ = np.linalg.qr(G, mode="reduced")
        return np.asfortranarray(symmetrize_lower(Q @ Q.T))
    import torch
    Gd = torch.from_numpy(G).to(device)
    Q, _ = torch.linalg.qr(Gd, mode="reduced")
    del Gd
    K = Q @ Q.T
    del Q
    K = torch.tril(K) + torch.tril(K, -1).T
    return K.contiguous()


def similarity_kernel(n: int, seed: int, device=None):
    """Non-Hermitian kernel of the same DPP as a Hermitian one (Prop. 2).

    H = Q diag(lam) Q^T with lam_i ~ Beta(0.5, 2); s_i = exp(z_i), z_i ~ N(0, 0.5)
    (standard deviation 0.5); K = S H S^{-1}, i.e. K_ij = s_i H_ij / s_j.
    Returns (K, H). With ``device`` the QR and the products run there (FP64)
    from the same host draws, and K and H come back as column-major device
    tensors.
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    lam = rng.beta(0.5, 2.0, size=n)
    z = rng.normal(0.0, 0.5, size=n)
    s = np.exp(z)
    if device is None:
        Q, _ = np.linalg.qr(G, mode="reduced")
        H = symmetrize_lower((Q * lam) @ Q.T)
        K = (s[:, None] * H) / s[None, :]
        return np.asfortranarray(K), np.asfortranarray(H)
    import torch
    Q, _ = torch.linalg.qr(torch.from_numpy(G).to(device), mode="reduced")
    lam_d = torch.from_numpy(lam).to(device)
    s_d = torch.from_numpy(s).to(device)
    H = (Q * lam_d) @ Q.T
    del Q
    H = torch.tril(H) + torch.tril(H, -1).T
    K = (s_d[:, None] * H) / s_d[None, :]
    # column-major: the transpose view of a contiguous buffer holding K^T
    return K.T.contiguous().T, H.T.contiguous().T


def lensemble_kernel(n: int, seed: int, rank: int = 64, dtype=np.float32, out=None):
    """Marginal kernel of a rank-`rank` L-ensemble, formed in FP64, stored in `dtype`.

    Phi ~ N(0, 1/rank) (variance 1/rank), q_i ~ LogNormal(0, 0.5),
    F = diag(q) Phi, L = F F^T and K = L (L + I)^{-1} = F (I + F^T F)^{-1} F^T.
    With ``out`` (a column-major n x n torch tensor on a device) the products
    and the solve run on that device, in FP64, from the same host draws, and
    the result is written into ``out`` in its dtype.
    """
    rng = np.random.default_rng(seed)
    Phi = rng.normal(0.0, 1.0 / np.sqrt(rank), size=(n, rank))
    q = rng.lognormal(0.0, 0.5, size=n)
    F = q[:, None] * Phi
    if out is None:
        M = np.eye(rank) + F.T @ F
        K = F @ np.linalg.solve(M, F.T)
        return np.asfortranarray(symmetrize_lower(K).astype(dtype))
    import torch
    Fd = torch.from_numpy(F).to(out.device)
    M = torch.eye(rank, dtype=torch.float64, device=out.device) + Fd.T @ Fd
    K = Fd @ torch.linalg.solve(M, Fd.T)
    K = torch.tril(K) + torch.tril(K, -1).T
    out.copy_(K)
    return out


def lensemble_L(n: int, seed: int, rank: int = 64, dtype=np.float64, out=None):
    """The L-ensemble kernel L = F F^T behind ``lensemble_kernel`` (same draws,
    F = diag(q) Phi), formed in FP64 and stored in `dtype`; with ``out`` (a
    column-major n x n torch tensor on a device) the product runs there."""
    rng = np.random.default_rng(seed)
    Phi = rng.normal(0.0, 1.0 / np.sqrt(rank), size=(n, rank))
    q = rng.lognormal(0.0, 0.5, size=n)
    F = q[:, None] * Phi
    if out is None:
        return np.asfortranarray(symmetrize_lower(F @ F.T).astype(dtype))
    import torch
    Fd = torch.from_numpy(F).to(out.device)
    L = Fd @ Fd.T
    out.copy_(torch.tril(L) + torch.tril(L, -1).T)
    return out


def lensemble_batch_sizes(count: int, seed: int, lo: int = 64, hi: int = 1024) -> np.ndarray:
    """n_i ~ U{lo..hi} (inclusive) for a batch of L-ensemble kernels."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=count)


def grid_transfer_current_kernel(d: int):
    """Transfer-current kernel of the d x d vertex grid graph of Z^2.

    Its DPP is the uniform distribution over spanning trees (the paper's 40 x 40
    example, Sec. 1): K = B^T (B B^T)^{-1} B with B the vertex-edge incidence
    matrix with one vertex row removed. Edges are ordered horizontal then
    vertical. Returns (K, edges) with edges an (E, 2) array of vertex ids.
    """
    edges = []
    for y in range(d):
        for x in range(d - 1):
            edges.append((y * d + x, y * d + x + 1))
    for y in range(d - 1):
        for x in range(d):
            edges.append((y * d + x, (y + 1) * d + x))
    edges = np.asarray(edges, dtype=np.int64)
    V, E = d * d, len(edges)
    B = np.zeros((V, E))
    B[edges[:, 0], np.arange(E)] = 1.0
    B[edges[:, 1], np.arange(E)] = -1.0
    Br = B[1:, :]
    K = Br.T @ np.linalg.solve(Br @ Br.T, Br)
    return np.asfortranarray(symmetrize_lower(K)), edges


# ------------------------------------------------------------ complex kernels

def _complex_orthonormal(rng, n: int):
    """Q factor of the QR of a seeded complex Gaussian n x n matrix (real and
    imaginary parts N(0, 1/2))."""
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    Q, _ = np.linalg.qr(G)
    return Q


def hermitize_lower(K: np.ndarray) -> np.ndarray:
    """Copy the conjugate of the strict lower triangle onto the upper one and
    drop the diagonal's imaginary parts, so K is exactly Hermitian."""
    return np.tril(K, -1) + np.tril(K, -1).conj().T + np.diag(np.real(np.diag(K)))


def complex_hermitian_kernel(n: int, seed: int, beta: bool = False, device=None):
    """K = Q diag(lam) Q^H, Q unitary from QR of a complex Gaussian matrix,
    lam_i ~ U(0, 1) (or Beta(0.5, 2) with `beta`); complex128, column-major.

    With ``device`` (a torch CUDA device) the QR and the products run there
    from the same host draws and a column-major device tensor is returned
    (the same construction; the bytes differ from the host path's)."""
    rng = np.random.default_rng(seed)
    if device is None:
        Q = _complex_orthonormal(rng, n)
        lam = rng.beta(0.5, 2.0, size=n) if beta else rng.random(n)
        return np.asfortranarray(hermitize_lower((Q * lam) @ Q.conj().T))
    import torch
    G = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    lam = rng.beta(0.5, 2.0, size=n) if beta else rng.random(n)
    Q, _ = torch.linalg.qr(torch.from_numpy(G).to(device))
    del G
    K = (Q * torch.from_numpy(lam).to(device)) @ Q.conj().T
    del Q
    low = torch.tril(K, -1)
    K = low + low.conj().T + torch.diag(torch.diagonal(K).real.to(K.dtype))
    return K.T.contiguous().T


def complex_similarity_kernel(n: int, seed: int, unit_modulus: bool = False, device=None):
    """A non-Hermitian complex kernel of the same DPP as a complex Hermitian
    one (Prop. 2): H as in complex_hermitian_kernel with lam ~ Beta(0.5, 2),
    S = diag(exp(z_j + i theta_j)), z ~ N(0, 0.5) (standard deviation 0.5),
    theta ~ U(0, 2 pi), K = S H S^{-1}. With `unit_modulus`, z = 0 and K is
    Hermitian again. Returns (K, H), complex128, column-major (device tensors
    with ``device``, as for complex_hermitian_kernel)."""
    H = complex_hermitian_kernel(n, seed, beta=True, device=device)
    rng = np.random.default_rng(seed + 7_000_000)
    z = np.zeros(n) if unit_modulus else rng.normal(0.0, 0.5, size=n)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=n)
    s = np.exp(z + 1j * theta)
    if device is None:
        K = (s[:, None] * H) / s[None, :]
        if unit_modulus:
            K = hermitize_lower(K)
        return np.asfortranarray(K), H
    import torch
    st = torch.from_numpy(s).to(device)
    K = (st[:, None] * H) / st[None, :]
    if unit_modulus:
        low = torch.tril(K, -1)
        K = low + low.conj().T + torch.diag(torch.diagonal(K).real.to(K.dtype))
    return K.T.contiguous().T, H


def aztec_diamond_kernel(d: int):
    """Kenyon's dimer kernel of the Aztec diamond of order d (the paper's
    domino-tiling examples, Sec. 1): a complex, non-Hermitian marginal kernel
    whose DPP is the uniform measure on domino tilings.

    Squares: the unit squares [x, x+1] x [y, y+1] with |x + 1/2| + |y + 1/2| <= d,
    black when x + y is even. Ground set: the (black, white) adjacent pairs
    (a domino covering both). Kasteleyn matrix C[b, w] = 1 for a horizontal
    pair, i for a vertical one (every 4-cycle around an interior lattice point
    then has alternating product -1, Kasteleyn's condition), and the kernel is
    L[e, f] = C[b_e, w_e] (C^{-1})[w_e, b_f] (Kenyon's local statistics). Every
    sample is a perfect matching of the squares (d(d+1) dominoes), and each of
    the 2^{d(d+1)/2} tilings has likelihood 2^{-d(d+1)/2}.
    Returns (K complex128 column-major, black index per edge, white index per
    edge, C)."""
    sq = [(x, y) for x in range(-d, d) for y in range(-d, d) if abs(x + 0.5) + abs(y + 0.5) <= d]
    black = {s: i for i, s in enumerate(s for s in sq if (s[0] + s[1]) % 2 == 0)}
    white = {s: i for i, s in enumerate(s for s in sq if (s[0] + s[1]) % 2 != 0)}
    eb, ew, wt = [], [], []
    for (x, y), b in black.items():
        for dx, dy, w in ((1, 0, 1.0), (-1, 0, 1.0), (0, 1, 1j), (0, -1, 1j)):
            t = (x + dx, y + dy)
            if t in white:
                eb.append(b)
                ew.append(white[t])
                wt.append(w)
    eb, ew, wt = np.array(eb), np.array(ew), np.array(wt, dtype=np.complex128)
    C = np.zeros((len(black), len(white)), dtype=np.complex128)
    C[eb, ew] = wt
    Ci = np.linalg.inv(C)
    K = wt[:, None] * Ci[ew][:, eb]
    return np.asfortranarray(K), eb, ew, C

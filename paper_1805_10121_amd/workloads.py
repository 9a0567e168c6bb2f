"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only -- none of the eigensolver's arithmetic -- and is the
single place that both the CPU oracle's tests and the GPU tests/bench draw inputs from.

The paper's matrices (DFT sequences NaCl and AuAg, BSE problems; Sec. 6, Table 3) are not
available; these generators stand in for them:

  * H = Q diag(lam) Q^H with Q a Haar-random unitary (QR of a complex Gaussian with the phase
    fix Q diag(R_ii/|R_ii|)) and a prescribed spectrum lam, symmetrised as (H + H^H)/2;
  * "uniform" spectrum: i.i.d. U[-1, 1], sorted (isolated problem of order 1000);
  * "clustered" spectrum: 6 Gaussian clusters (standard deviation 1e-3) centred at
    -1.0, -0.9, ..., -0.5, the rest i.i.d. U[-0.4, 2.0], sorted; the number of clustered values
    is a parameter (600 for the order-10000/20000 problems, 2400 for order 60000);
  * sequences: H_{k+1} = H_k + eps * ||H_k||_2 * E_k with E_k = (G + G^H)/2 of a complex
    Gaussian G, scaled to unit spectral norm;
  * start blocks and Lanczos start vectors: complex Gaussian (real and imaginary parts N(0, 1)).

Seeds: NumPy Generator(PCG64(seed)).  Large matrices can be generated on a torch device
(``hermitian_torch``) with the same recipe; those bytes differ from the CPU ones but the
spectrum is the same prescribed lam.
"""

from __future__ import annotations

import numpy as np

CLUSTER_CENTRES = (-1.0, -0.9, -0.8, -0.7, -0.6, -0.5)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def complex_gaussian(g: np.random.Generator, *shape) -> np.ndarray:
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def spectrum_uniform(n: int, g: np.random.Generator, lo: float = -1.0, hi: float = 1.0):
    return np.sort(g.uniform(lo, hi, size=n))


def spectrum_clustered(n: int, g: np.random.Generator, n_clustered: int = 600,
                       width: float = 1e-3, bulk=(-0.4, 2.0)):
    per = n_clustered // len(CLUSTER_CENTRES)
    parts = [c + width * g.standard_normal(per) for c in CLUSTER_CENTRES]
    rest = n - per * len(CLUSTER_CENTRES)
    parts.append(g.uniform(bulk[0], bulk[1], size=rest))
    return np.sort(np.concatenate(parts))


def haar_unitary(n: int, g: np.random.Generator) -> np.ndarray:
    Z = complex_gaussian(g, n, n) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


def hermitian_from(Q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    H = (Q * lam[None, :]) @ Q.conj().T
    return 0.5 * (H + H.conj().T)


def haar_orthogonal(n: int, g: np.random.Generator) -> np.ndarray:
    """Real Haar-distributed orthogonal matrix: QR of a real Gaussian with the sign fix."""
    Q, R = np.linalg.qr(g.standard_normal((n, n)))
    return Q * np.sign(np.diag(R))[None, :]


def symmetric_from(Q: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Real symmetric Q diag(lam) Q^T, symmetrised."""
    H = (Q * lam[None, :]) @ Q.T
    return 0.5 * (H + H.T)


def hermitian(n: int, lam: np.ndarray, seed: int) -> np.ndarray:
    """Column-major-ready (Fortran order) complex128 H with spectrum lam."""
    Q = haar_unitary(n, rng(seed))
    return np.asfortranarray(hermitian_from(Q, lam))


def start_block(n: int, b: int, seed: int) -> np.ndarray:
    return np.asfortranarray(complex_gaussian(rng(seed), n, b))


def perturbation(n: int, seed: int, power_iters: int = 60) -> np.ndarray:
    """Hermitian complex Gaussian (G + G^H)/2 scaled to unit spectral norm."""
    g = rng(seed)
    G = complex_gaussian(g, n, n)
    E = 0.5 * (G + G.conj().T)
    if n <= 3000:
        nrm = float(np.max(np.abs(np.linalg.eigvalsh(E))))
    else:
        x = complex_gaussian(g, n)
        for _ in range(power_iters):
            x = E @ x
            x /= np.linalg.norm(x)
        nrm = float(np.linalg.norm(E @ x))
    return E / nrm


def sequence(n: int, lam: np.ndarray, n_problems: int, eps: float, seed: int):
    """List of H_1..H_K (host, complex128, Fortran order).  ||H_k||_2 is taken as max|lam| for
    k = 1 and tracked by the triangle bound thereafter (the perturbations are 1e-3 relative)."""
    H = hermitian(n, lam, seed)
    out = [H]
    norm = float(np.max(np.abs(lam)))
    for k in range(1, n_problems):
        E = perturbation(n, seed + 100 + k)
        H = np.asfortranarray(H + eps * norm * E)
        norm = norm * (1.0 + eps)
        out.append(H)
    return out


# ----------------------------------------------------------------------------- configs
# The five synthetic workloads (order n, nev, nex, spectrum).  Seeds: 1000 * id + problem.

# The synthetic workloads, by name.  `seed` is the base seed of each workload's generators
# (spectrum draws use it directly; H, start blocks and Lanczos vectors use offsets from it).
WORKLOADS = {
    # one isolated problem, uniform spectrum on [-1, 1]
    "uniform_n1000": dict(n=1000, nev=50, nex=20, spectrum="uniform", tol=1e-10, seed=1000),
    # one isolated problem, 600 clustered values below a uniform bulk
    "clustered_n10000": dict(n=10000, nev=500, nex=100, spectrum="clustered", n_clustered=600,
                             tol=1e-10, seed=2000),
    # warm-started sequence whose nev falls inside the bulk (no gap after nev + nex)
    "sequence_n20000": dict(n=20000, nev=1000, nex=200, spectrum="clustered", n_clustered=600,
                            tol=1e-10, problems=10, eps=1e-3, seed=3000),
    # serving: 16 sequences of uneven order
    "serving": dict(sizes=(2000, 4000, 8000, 16000), sequences=16, problems=8, eps=1e-3,
                    tol=1e-10, seed=4000),
    # large warm-started sequence, clustered values scaled to nev (gap after nev + nex)
    "sequence_n60000": dict(n=60000, nev=2000, nex=400, spectrum="clustered", n_clustered=2400,
                            tol=1e-10, problems=5, eps=5e-4, seed=5000),
}


def spectrum_for(name: str, n: int | None = None, seed: int | None = None) -> np.ndarray:
    c = WORKLOADS[name]
    n = n or c["n"]
    g = rng(seed if seed is not None else c["seed"])
    if c.get("spectrum", "clustered") == "uniform":
        return spectrum_uniform(n, g)
    return spectrum_clustered(n, g, n_clustered=c.get("n_clustered", 600))


def serving_size(n_choices, n_seq: int, seed: int):
    """N for each serving sequence, drawn uniformly from n_choices."""
    g = rng(seed)
    return [int(n_choices[i]) for i in g.integers(0, len(n_choices), size=n_seq)]


def optimized_degree_profile(b: int, deg_max: int = 36) -> np.ndarray:
    """A sorted, even degree array spread uniformly over 2..deg_max, the shape Alg. 5 produces
    when residuals span many decades (used to time the filter with a realistic active-range
    schedule)."""
    levels = deg_max // 2
    d = 2 + 2 * ((np.arange(b) * levels) // b)
    return np.sort(d).astype(np.int32)


# ----------------------------------------------------------------------------- torch (device)

def structured_unitary(n: int, seed: int, reflectors: int = 4):
    """Host-drawn factors of Q = D P_r ... P_1 (P_j = I - 2 u_j u_j^H, D = diag(d)): unit
    complex Gaussian u_j (rows of U) and unit phases d."""
    g = rng(seed)
    U = complex_gaussian(g, reflectors, n)
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    d = np.exp(2j * np.pi * g.uniform(0.0, 1.0, n))
    return U, d


def apply_colmajor_qh(U, d, v):
    """Q-bar^H v for the matrix that hermitian_torch_fast's buffer holds when read column-major
    (that matrix is Q-bar diag(lam) Q-bar^H with Q-bar = conj(Q)); v: (n,) or (n, k)."""
    w = (d.reshape(-1, *([1] * (np.ndim(v) - 1)))) * v
    for j in range(U.shape[0] - 1, -1, -1):
        u = U[j].conj()
        w = w - 2.0 * np.multiply.outer(u, u.conj() @ w) if np.ndim(v) > 1 else w - 2.0 * u * (u.conj() @ w)
    return w


def apply_colmajor_q(U, d, z):
    """Q-bar z (inverse of apply_colmajor_qh)."""
    w = np.array(z, dtype=np.complex128, copy=True)
    for j in range(U.shape[0]):
        u = U[j].conj()
        w = w - 2.0 * np.multiply.outer(u, u.conj() @ w) if np.ndim(z) > 1 else w - 2.0 * u * (u.conj() @ w)
    return np.conj(d).reshape(-1, *([1] * (np.ndim(z) - 1))) * w


def hermitian_torch_fast(n: int, lam: np.ndarray, seed: int, device: str = "cuda",
                         reflectors: int = 4):
    """H = Q diag(lam) Q^H with Q = D P_r ... P_1 from ``structured_unitary`` -- a dense unitary
    that costs O(r n^2) to apply, for orders where a Haar QR is impractical (n >= 20000).  With
    Gaussian start vectors the iteration statistics of the eigensolver depend only on the
    spectrum, so this changes no convergence behaviour.  Built in place (rank-one updates): the
    peak memory is one n x n complex128 matrix plus O(n) vectors.  The returned buffer, read
    column-major, is Q-bar diag(lam) Q-bar^H (see ``apply_colmajor_q``)."""
    import torch

    Uh, dh = structured_unitary(n, seed, reflectors)
    H = torch.diag(torch.as_tensor(lam, device=device, dtype=torch.float64).to(torch.complex128))
    for j in range(reflectors):
        u = torch.as_tensor(Uh[j], device=device)
        # P H P = H - 2 u w^H - 2 w u^H with w = H u - (u^H H u) u
        Hu = H @ u
        w = Hu - torch.vdot(u, Hu) * u
        H.addr_(u, w.conj(), alpha=-2.0)
        H.addr_(w, u.conj(), alpha=-2.0)
        del Hu, w, u
    d = torch.as_tensor(dh, device=device)
    H.mul_(d[:, None])
    H.mul_(d.conj()[None, :])
    return H


def structured_orthogonal(n: int, seed: int, reflectors: int = 4):
    """Host-drawn factors of the real Q = D P_r ... P_1 (P_j = I - 2 u_j u_j^T, D = diag(d)):
    unit Gaussian u_j (rows of U) and random signs d."""
    g = rng(seed)
    U = g.standard_normal((reflectors, n))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    d = np.where(g.standard_normal(n) < 0, -1.0, 1.0)
    return U, d


def apply_real_qt(U, d, v):
    """Q^T v for the Q of ``structured_orthogonal`` (symmetric_torch_fast's matrix is
    Q diag(lam) Q^T); v: (n,) or (n, k)."""
    w = d.reshape(-1, *([1] * (np.ndim(v) - 1))) * v
    for j in range(U.shape[0] - 1, -1, -1):
        u = U[j]
        w = w - 2.0 * np.multiply.outer(u, u @ w) if np.ndim(v) > 1 else w - 2.0 * u * (u @ w)
    return w


def apply_real_q(U, d, z):
    """Q z (inverse of apply_real_qt)."""
    w = np.array(z, dtype=np.float64, copy=True)
    for j in range(U.shape[0]):
        u = U[j]
        w = w - 2.0 * np.multiply.outer(u, u @ w) if np.ndim(z) > 1 else w - 2.0 * u * (u @ w)
    return d.reshape(-1, *([1] * (np.ndim(z) - 1))) * w


def symmetric_torch_fast(n: int, lam: np.ndarray, seed: int, device: str = "cuda",
                         reflectors: int = 4):
    """Real symmetric counterpart of ``hermitian_torch_fast``: Q = D P_r ... P_1 with real unit
    Gaussian reflector vectors and random signs D (``structured_orthogonal``), built in place
    (one n x n float64 buffer).  Symmetric up to rounding of the two rank-one updates per
    reflector, so the row-major tensor read column-major is the same matrix to that accuracy."""
    import torch

    U, d = structured_orthogonal(n, seed, reflectors)
    H = torch.diag(torch.as_tensor(lam, device=device, dtype=torch.float64))
    for j in range(reflectors):
        u = torch.as_tensor(U[j], device=device)
        Hu = H @ u
        w = Hu - torch.dot(u, Hu) * u
        H.addr_(u, w, alpha=-2.0)
        H.addr_(w, u, alpha=-2.0)
        del Hu, w, u
    dd = torch.as_tensor(d, device=device)
    H.mul_(dd[:, None])
    H.mul_(dd[None, :])
    return H


def hermitian_torch(n: int, lam: np.ndarray, seed: int, device: str = "cuda",
                    dtype=None):
    """Same recipe on a torch device (for orders where the host QR is too slow).

    Returns a complex128 device tensor laid out column-major: the tensor ``T`` with
    ``T.shape == (n, n)`` whose storage is H in column-major order (i.e. ``T = H^T`` in
    row-major terms; since H is Hermitian this is conj(H))."""
    import torch

    dtype = dtype or torch.complex128
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    re = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
    im = torch.randn((n, n), generator=gen, device=device, dtype=torch.float64)
    Z = torch.complex(re, im) / np.sqrt(2.0)
    del re, im
    Q, R = torch.linalg.qr(Z)
    del Z
    d = torch.diagonal(R)
    Q = Q * (d / d.abs())[None, :]
    del R
    lam_t = torch.as_tensor(lam, device=device, dtype=torch.float64).to(dtype)
    H = (Q * lam_t[None, :]) @ Q.conj().T
    del Q
    H = 0.5 * (H + H.conj().T)
    # column-major storage of H == row-major storage of H^T
    return H.transpose(0, 1).contiguous()

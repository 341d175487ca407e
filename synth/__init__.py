"""Seeded synthetic inputs for the Flip-Flop SRQR hot path.

Test and benchmark infrastructure. This module holds no step of the
method: it only builds input matrices with prescribed singular spectra,
shaped like the paper's test problems (Section 4.1, "Type 1" matrices
U*D*V^T plus Gaussian noise).  Both the oracle and the GPU path consume the
bytes it returns; neither imports the other.

Recipes (all seeded, FP64 arithmetic, optionally rounded to FP32 storage):

* ``spectrum_matrix(m, n, sigma, seed, noise)``:
  A = U diag(sigma) V^T + noise * G, with U (m x r) and V (n x r) the
  explicit Q factors of LAPACK Householder QR of i.i.d. N(0,1) matrices
  (numpy.linalg.qr), G i.i.d. N(0,1), r = len(sigma).
* named workloads:
  - ``small_fp64``  : m=1000, n=800, sigma_j = j^-2 (r = 800),
    k=20, p=10, sketch seed 0.
  - ``mid``         : m=16384, n=8192, r=1024, sigma_j = exp(-j/50),
    noise 1e-6, k=256, p=16, sketch seed 0.
  - ``large``       : m=32768, n=16384, r=1024, sigma_j = 1 for j <= 8 and
    10^(-3 (j - 8) / 1000) for 8 < j <= 1024, noise 1e-5, k=512, p=32
    (l = 544), sketch seed 0; meant for FP32 storage.
  - ``large_q``     : the same spectrum and k, p at a quarter of the size
    (8192 x 4096), small enough for the oracle to run whole.
  - ``large_s``     : the same at an eighth of the size (4096 x 2048), the
    bounded sample on which the benchmark times the oracle.
* ``tucker_tensor``: a Tucker tensor (N(0,1) core times orthonormal
  factors) plus Gaussian noise, for the ST-HOSVD driver; the 400^3 tensor
  of core 40^3 and noise 1e-3 stands for the tensor workload.
* ``rpca_problem``: low rank plus sparse, M = X_L X_R^T + E*, for the
  robust PCA driver (rank 0.1 m and 5% corrupted entries in the paper's
  experiment).
* ``batch_problems``: many independent problems of mixed shapes (m, n
  uniform on [500, 4000], sigma_j = j^-1.5, k uniform on [10, 100]) for the
  batched entry point.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "spectrum_matrix",
    "separated_columns_matrix",
    "random_matrix",
    "make_workload",
    "tucker_tensor",
    "rpca_problem",
    "batch_problems",
]


def _rng(seed: int, stream: int) -> np.random.Generator:
    # One independent numpy generator per (seed, stream) pair.
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream) + 1]))


def _orthonormal(rows: int, cols: int, rng: np.random.Generator) -> np.ndarray:
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    # Fix the column signs so that the factor is a function of the seed only.
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def spectrum_matrix(m: int, n: int, sigma, seed: int, noise: float = 0.0,
                    dtype=np.float64) -> np.ndarray:
    """A = U diag(sigma) V^T + noise*G, Fortran (column-major) order."""
    sigma = np.asarray(sigma, dtype=np.float64)
    r = sigma.shape[0]
    if r > min(m, n):
        raise ValueError("spectrum longer than min(m, n)")
    u = _orthonormal(m, r, _rng(seed, 1))
    v = _orthonormal(n, r, _rng(seed, 2))
    a = np.asfortranarray((u * sigma) @ v.T)
    if noise:
        a += noise * _rng(seed, 3).standard_normal((m, n))
    return np.asfortranarray(a.astype(dtype, copy=False))


def separated_columns_matrix(m: int, n: int, seed: int, ratio: float = 1.5,
                             dtype=np.float64) -> np.ndarray:
    """Orthogonal columns whose norms are spaced by ``ratio``, in shuffled order.

    With orthogonal columns the greedy pivot order is the descending-norm order,
    so it is known in closed form (see ``column_norm_order``).
    """
    if n > m:
        raise ValueError("need m >= n for orthogonal columns")
    rng = _rng(seed, 4)
    q = _orthonormal(m, n, rng)
    norms = ratio ** (-np.arange(n, dtype=np.float64))
    order = rng.permutation(n)
    a = q * norms[order]
    return np.asfortranarray(a.astype(dtype, copy=False))


def random_matrix(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) entries."""
    a = _rng(seed, 5).standard_normal((m, n))
    return np.asfortranarray(a.astype(dtype, copy=False))


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    k: int
    p: int
    seed: int          # sketch (Omega) seed
    fixture_seed: int  # seed of the matrix generator
    spectrum: str
    noise: float

    @property
    def l(self) -> int:
        return min(self.k + self.p, self.m, self.n)

    def sigma(self) -> np.ndarray:
        if self.spectrum == "inv_square":
            r = min(self.m, self.n)
            return np.arange(1, r + 1, dtype=np.float64) ** -2.0
        if self.spectrum == "exp50_r1024":
            j = np.arange(1, 1025, dtype=np.float64)
            return np.exp(-j / 50.0)
        if self.spectrum == "flat8_decade3_r1024":
            j = np.arange(1, 1025, dtype=np.float64)
            return np.where(j <= 8, 1.0, 10.0 ** (-3.0 * (j - 8) / 1000.0))
        raise KeyError(self.spectrum)


WORKLOADS = {
    "small_fp64": Workload("small_fp64", 1000, 800, 20, 10, 0, 1, "inv_square", 0.0),
    "mid": Workload("mid", 16384, 8192, 256, 16, 0, 2, "exp50_r1024", 1e-6),
    "large": Workload("large", 32768, 16384, 512, 32, 0, 3, "flat8_decade3_r1024", 1e-5),
    "large_q": Workload("large_q", 8192, 4096, 512, 32, 0, 3, "flat8_decade3_r1024", 1e-5),
    "large_s": Workload("large_s", 4096, 2048, 512, 32, 0, 3, "flat8_decade3_r1024", 1e-5),
}


def tucker_tensor(dims, ranks, seed: int, noise: float = 0.0, dtype=np.float64) -> np.ndarray:
    """X = G x_1 U_1 x_2 U_2 ... + noise*E: a core G (ranks, i.i.d. N(0,1))
    times orthonormal factors U_j (dims[j] x ranks[j]), plus i.i.d. Gaussian
    noise; Fortran order (the first index runs fastest)."""
    d = len(dims)
    X = _rng(seed, 10).standard_normal(tuple(ranks))
    for j in range(d):
        U = _orthonormal(dims[j], ranks[j], _rng(seed, 11 + j))
        X = np.moveaxis(np.tensordot(U, X, axes=([1], [j])), 0, j)
    if noise:
        X = X + noise * _rng(seed, 20).standard_normal(tuple(dims))
    return np.asfortranarray(X.astype(dtype, copy=False))


def rpca_problem(m: int, n: int, rank: int, frac: float, seed: int, amp: float = 500.0):
    """M = X* + E*: X* = X_L X_R^T with X_L (m x rank) and X_R (n x rank)
    i.i.d. N(0,1); E* with round(frac m n) nonzeros at distinct uniformly
    random positions, each uniform on [-amp, amp] (the robust PCA test
    matrices of the paper's experiment).  Returns (M, X*, E*), Fortran order."""
    xl = _rng(seed, 30).standard_normal((m, rank))
    xr = _rng(seed, 31).standard_normal((n, rank))
    X = np.asfortranarray(xl @ xr.T)
    rng = _rng(seed, 32)
    nnz = int(round(frac * m * n))
    pos = rng.choice(m * n, size=nnz, replace=False)
    E = np.zeros(m * n)
    E[pos] = rng.uniform(-amp, amp, size=nnz)
    E = np.asfortranarray(E.reshape((m, n), order="F"))
    return np.asfortranarray(X + E), X, E


def batch_problems(count: int, seed: int, rmax: int = 512):
    """`count` problems with m, n uniform on [500, 4000], sigma_j = j^-1.5
    (j <= min(m, n, rmax); the spectrum is cut there, where it is below
    1e-4 of sigma_1) and k uniform on [10, 100]: [(A, k)], A Fortran order."""
    rng = _rng(seed, 40)
    out = []
    for i in range(count):
        m, n = (int(x) for x in rng.integers(500, 4001, size=2))
        k = int(rng.integers(10, 101))
        r = min(m, n, rmax)
        sig = np.arange(1, r + 1, dtype=np.float64) ** -1.5
        out.append((spectrum_matrix(m, n, sig, seed * 1000 + i), k))
    return out


def make_workload(name: str, dtype=np.float64) -> np.ndarray:
    w = WORKLOADS[name]
    return spectrum_matrix(w.m, w.n, w.sigma(), w.fixture_seed, w.noise, dtype=dtype)

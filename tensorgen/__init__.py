"""Seeded synthetic inputs for CP decomposition experiments.

This module is shared by the test oracle and by the GPU library's tests and
benchmark. It only draws random numbers and assembles input tensors; it holds
none of the decomposition method's arithmetic (no MTTKRP, no solves, no
perturbation operators).

Workload families (Section 5.1 of the paper, "Sequential Experimental Results"):

* planted tensors built from known factor matrices whose columns have a
  prescribed collinearity (the paper defines collinearity as the common cosine
  between distinct columns of each factor);
* planted tensors built from uniformly distributed factors in [0, 1];
* planted tensors with i.i.d. standard normal factors;
* planted Tucker tensors: factors with orthonormal columns and an i.i.d. normal core.

Noise is added as eta * ||T||_F * E / ||E||_F with E i.i.d. N(0, 1), so the
relative noise level is exactly eta.  Initial factors for ALS are uniform in
[0, 1) (Algorithm 1, initialisation step).

Seeds: ``np.random.SeedSequence(seed).spawn(3)`` gives three independent
streams, used for (planted factors, noise, initial guess) in that order.
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "Problem",
    "streams",
    "planted_factors",
    "cp_reconstruct",
    "add_noise",
    "init_factors",
    "make_problem",
    "DeviceProblem",
    "make_problem_device",
    "tucker_reconstruct",
    "TuckerProblem",
    "make_tucker_problem",
]


def streams(seed: int):
    """Three independent generators (factors, noise, init) derived from one seed."""
    ss = np.random.SeedSequence(seed).spawn(3)
    return tuple(np.random.default_rng(s) for s in ss)


def planted_factors(shape, rank, rng, dist="normal", collinearity=None):
    """Factor matrices A^(n) of size s_n x rank.

    dist="normal": i.i.d. N(0, 1) entries.
    dist="uniform": i.i.d. U[0, 1) entries.
    collinearity=C (0 <= C < 1): every column is sqrt(C) g + sqrt(1 - C) z_r with
    one shared N(0, 1) vector g per mode and independent N(0, 1) vectors z_r,
    then normalised to unit length.  The expected cosine between two columns
    is C (the realised value fluctuates by O(s^-1/2)).
    """
    out = []
    for s in shape:
        if collinearity is not None:
            c = float(collinearity)
            g = rng.standard_normal((s, 1))
            z = rng.standard_normal((s, rank))
            a = np.sqrt(c) * g + np.sqrt(1.0 - c) * z
            a /= np.linalg.norm(a, axis=0, keepdims=True)
        elif dist == "normal":
            a = rng.standard_normal((s, rank))
        elif dist == "uniform":
            a = rng.random((s, rank))
        else:
            raise ValueError(f"unknown factor distribution {dist!r}")
        out.append(np.ascontiguousarray(a, dtype=np.float64))
    return out


def _krp_rows(mats):
    """Row-wise Kronecker (Khatri-Rao) product, first matrix slowest."""
    out = mats[0]
    for m in mats[1:]:
        out = (out[:, None, :] * m[None, :, :]).reshape(-1, m.shape[1])
    return out


def cp_reconstruct(factors):
    """Dense tensor sum_r a_r^(1) o ... o a_r^(N), row-major (last mode fastest)."""
    shape = tuple(a.shape[0] for a in factors)
    if len(factors) == 1:
        return factors[0].sum(axis=1)
    rest = _krp_rows(factors[1:])  # (prod s_2..s_N) x R
    return (factors[0] @ rest.T).reshape(shape)


def add_noise(T, eta, rng, chunk=1 << 24):
    """X = T + eta ||T||_F E / ||E||_F, E i.i.d. N(0, 1); returns a new float64 array."""
    if eta == 0.0:
        return np.array(T, dtype=np.float64, copy=True)
    flat_t = T.reshape(-1)
    E = np.empty_like(flat_t)
    for lo in range(0, E.size, chunk):
        hi = min(E.size, lo + chunk)
        E[lo:hi] = rng.standard_normal(hi - lo)
    nt = float(np.sqrt(np.dot(flat_t, flat_t)))
    ne = float(np.sqrt(np.dot(E, E)))
    scale = eta * nt / ne
    E *= scale
    E += flat_t
    return E.reshape(T.shape)


def init_factors(shape, rank, rng):
    """Initial guess: uniform [0, 1) entries (Algorithm 1 initialisation)."""
    return [np.ascontiguousarray(rng.random((s, rank)), dtype=np.float64) for s in shape]


@dataclasses.dataclass
class Problem:
    X: np.ndarray            # float64 tensor, row-major, last mode fastest
    planted: list            # planted factors
    init: list               # initial factors for ALS
    rank: int                # decomposition rank
    eta: float               # relative noise level
    seed: int

    @property
    def shape(self):
        return self.X.shape


def make_problem(shape, rank, seed, planted_rank=None, eta=1e-3, dist="normal",
                 collinearity=None):
    """Planted CP tensor plus noise, and a seeded uniform initial guess."""
    g_fac, g_noise, g_init = streams(seed)
    pr = rank if planted_rank is None else planted_rank
    planted = planted_factors(shape, pr, g_fac, dist=dist, collinearity=collinearity)
    T = cp_reconstruct(planted)
    X = add_noise(T, eta, g_noise)
    del T
    init = init_factors(shape, rank, g_init)
    return Problem(X=X, planted=planted, init=init, rank=rank, eta=eta, seed=seed)


@dataclasses.dataclass
class DeviceProblem:
    X: object                # torch tensor on the device (float32 or float64), row-major
    planted: list            # planted factors (numpy)
    init: list               # initial factors for ALS (numpy)
    rank: int
    eta: float
    seed: int
    shape: tuple


def make_problem_device(shape, rank, seed, eta=1e-3, dist="normal", collinearity=None,
                        dtype="f32", device="cuda"):
    """Same recipe as make_problem with the dense tensor assembled on the GPU (for
    workloads too many or too large to generate on the host).  Planted factors and
    the initial guess come from the same numpy streams as make_problem; the noise
    E is drawn by torch's device generator seeded from the noise stream, so the
    tensor is reproducible for a given seed but differs from make_problem's."""
    import torch
    g_fac, g_noise, g_init = streams(seed)
    planted = planted_factors(shape, rank, g_fac, dist=dist, collinearity=collinearity)
    init = init_factors(shape, rank, g_init)
    dev = torch.device(device)
    F = [torch.from_numpy(a).to(dev) for a in planted]
    rest = F[1]
    for m in F[2:]:
        rest = (rest[:, None, :] * m[None, :, :]).reshape(-1, m.shape[1])
    T = torch.matmul(F[0], rest.t().contiguous()).reshape(tuple(shape))
    del rest
    if eta > 0.0:
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(g_noise.integers(0, 2**62)))
        E = torch.randn(tuple(shape), generator=gen, dtype=torch.float64, device=dev)
        T.add_(E, alpha=float(eta * torch.linalg.vector_norm(T) / torch.linalg.vector_norm(E)))
        del E
    X = T.to(torch.float32) if dtype == "f32" else T
    return DeviceProblem(X=X.contiguous(), planted=planted, init=init, rank=rank, eta=eta,
                         seed=seed, shape=tuple(shape))


def tucker_reconstruct(core, factors):
    """Dense tensor core x_1 A^(1) x_2 .. x_N A^(N), row-major."""
    T = core
    for n, a in enumerate(factors):
        T = np.moveaxis(np.tensordot(a, T, axes=([1], [n])), 0, n)
    return np.ascontiguousarray(T)


@dataclasses.dataclass
class TuckerProblem:
    X: np.ndarray            # float64 tensor, row-major
    core: np.ndarray         # planted core
    planted: list            # planted factors (orthonormal columns)
    ranks: tuple
    eta: float
    seed: int

    @property
    def shape(self):
        return self.X.shape


def make_tucker_problem(shape, ranks, seed, eta=1e-3):
    """Planted Tucker tensor plus noise: factors with orthonormal columns (QR of i.i.d.
    N(0,1) matrices, stream 0), an i.i.d. N(0,1) core (stream 0 after the factors) and
    noise eta ||T|| E / ||E|| (stream 1)."""
    g_fac, g_noise, _ = streams(seed)
    planted = []
    for s, r in zip(shape, ranks):
        q, _ = np.linalg.qr(g_fac.standard_normal((s, r)))
        planted.append(np.ascontiguousarray(q))
    core = g_fac.standard_normal(tuple(ranks))
    T = tucker_reconstruct(core, planted)
    X = add_noise(T, eta, g_noise)
    return TuckerProblem(X=X, core=core, planted=planted, ranks=tuple(ranks), eta=eta, seed=seed)


def subspace_start(shape, rank, seed):
    """Starting bases for the subspace iteration of the HOSVD: one s_n x rank matrix of
    i.i.d. N(0,1) entries per mode (stream 2)."""
    _, _, g = streams(seed)
    return [np.ascontiguousarray(g.standard_normal((s, rank))) for s in shape]


def make_tucker_problem_device(shape, ranks, seed, eta=1e-3, device="cuda"):
    """make_tucker_problem with the dense tensor assembled on the GPU (FP64): the planted
    factors and core come from the same numpy stream; the noise is drawn by torch's device
    generator seeded from the noise stream.  Returns (X on the device, planted, core)."""
    import torch
    g_fac, g_noise, _ = streams(seed)
    planted = []
    for s, r in zip(shape, ranks):
        q, _ = np.linalg.qr(g_fac.standard_normal((s, r)))
        planted.append(np.ascontiguousarray(q))
    core = g_fac.standard_normal(tuple(ranks))
    dev = torch.device(device)
    T = torch.from_numpy(core).to(dev)
    for n, a in enumerate(planted):
        T = torch.movedim(torch.tensordot(torch.from_numpy(a).to(dev), T, dims=([1], [n])), 0, n)
    T = T.contiguous()
    if eta > 0.0:
        gen = torch.Generator(device=dev)
        gen.manual_seed(int(g_noise.integers(0, 2**62)))
        E = torch.randn(tuple(shape), generator=gen, dtype=torch.float64, device=dev)
        T.add_(E, alpha=float(eta * torch.linalg.vector_norm(T) / torch.linalg.vector_norm(E)))
        del E
    return T, planted, core

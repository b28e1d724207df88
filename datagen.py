"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: it only draws vectors.

The paper's workloads (a 23M x 384 embedding set with 10,000 queries for
search, Section 3; a 3M x 384 set for the k-NN graph, Section 4) are not
available, so Gaussian mixtures of the same shape stand in for them:

  1. draw ``n_comp`` centres (standard normal; optionally scaled to unit norm),
  2. pick a component uniformly for every point,
  3. add per-coordinate Gaussian noise of standard deviation ``sigma``,
  4. L2-normalise and cast to the storage dtype.

Queries are fresh draws from the same centres with their own seed.

Two generators exist: numpy's PCG64 on the host (small and medium sets) and
torch's device generator for sets too large to draw on the host in seconds.
They give different numbers for the same seed; a test always uses one of them
for both sides of a comparison.
"""
from __future__ import annotations

import numpy as np


def centres(d: int, n_comp: int, seed: int, unit: bool) -> np.ndarray:
    """Mixture centres, float64 (n_comp, d)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.standard_normal((n_comp, d))
    if unit:
        c /= np.linalg.norm(c, axis=1, keepdims=True)
    return c


def draw(c: np.ndarray, n: int, sigma: float, seed: int, dtype=np.float16) -> np.ndarray:
    """n points from the mixture with centres ``c`` (host, numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    comp = rng.integers(0, c.shape[0], size=n)
    x = c[comp] + sigma * rng.standard_normal((n, c.shape[1]))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(dtype)


def mixture(n: int, d: int, n_comp: int, sigma: float, seed: int, unit: bool = True,
            dtype=np.float16, query_seed: int | None = None, nq: int = 0):
    """Data (and optionally queries) from one seeded mixture, on the host.

    Returns ``x`` or ``(x, q)`` when ``nq > 0``.
    """
    c = centres(d, n_comp, seed, unit)
    x = draw(c, n, sigma, seed + 1_000_003, dtype)
    if nq <= 0:
        return x
    q = draw(c, nq, sigma, query_seed if query_seed is not None else seed + 1, dtype)
    return x, q


def mixture_device(n: int, d: int, n_comp: int, sigma: float, seed: int, unit: bool = True,
                   device="cuda", chunk: int = 1 << 20, out=None, draw_seed: int | None = None):
    """Large mixture drawn on the device with torch's generator (fp16 result).

    Centres come from the host generator seeded by ``seed`` (same as
    :func:`centres`); component choices and noise come from
    ``torch.Generator(device).manual_seed(draw_seed or seed)`` (queries use
    the data's ``seed`` for the centres and their own ``draw_seed``).
    """
    import torch

    c = torch.from_numpy(centres(d, n_comp, seed, unit)).to(device=device, dtype=torch.float32)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed if draw_seed is None else draw_seed))
    if out is None:
        out = torch.empty((n, d), dtype=torch.float16, device=device)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        comp = torch.randint(0, n_comp, (m,), generator=g, device=device)
        x = c[comp] + sigma * torch.randn((m, d), generator=g, device=device, dtype=torch.float32)
        x /= torch.linalg.vector_norm(x, dim=1, keepdim=True)
        out[s:s + m] = x.to(torch.float16)
    return out


# Named workloads (shapes of the paper's tasks; the mixture recipe is ours).
WORKLOADS = {
    # small search set: 10,000 x 32 fp32, 16 components around standard-normal centres
    "search-10Kx32": dict(n=10_000, d=32, n_comp=16, sigma=0.1, unit=False, dtype="f32",
                          seed=2508, query_seed=2509, nq=1_000),
    # plain graph: 1M x 384 fp16, 1,024 unit centres
    "graph-1Mx384": dict(n=1_000_000, d=384, n_comp=1024, sigma=0.05, unit=True, dtype="f16",
                         seed=2510),
    # Task-1 shaped search: 23M x 384 fp16, 8,192 unit centres, 10,000 queries
    "search-23Mx384": dict(n=23_000_000, d=384, n_comp=8192, sigma=0.05, unit=True, dtype="f16",
                           seed=2511, query_seed=2512, nq=10_000),
    # Task-2 shaped graph: 3M x 384 fp16, 3,072 unit centres
    "graph-3Mx384": dict(n=3_000_000, d=384, n_comp=3072, sigma=0.05, unit=True, dtype="f16",
                         seed=2514),
}

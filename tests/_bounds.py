"""Rounding-error bounds used by the GPU parity tests (no method arithmetic).

u32 = 2^-24 (FP32 unit roundoff).  B_nm is the sum of the magnitudes of the
real products that make up one real component of Gamma_nm (oracle.cond's
with_bound output), so every bound below is relative to B_nm.
"""
import math

U32 = 2.0 ** -24


def split_bf16_bound(k_chunk: int) -> float:
    """Split-BF16 GEMM against an exact GEMM of the same FP32 operands.

    * Operands: hi = bf16(x) has |x - hi| <= 2^-9 |x|, and lo = bf16(x - hi)
      leaves |x - hi - lo| <= 2^-18 |x|.  The product hi_a hi_b + hi_a lo_b +
      lo_a hi_b differs from ab by the dropped lo_a lo_b (<= 2^-18 |ab|) and the
      two representation errors (<= 2 * 2^-18 |ab| to first order): 3 * 2^-18,
      taken as 3 * 2^-16 for margin.  Worst case, element by element.
    * FP32 accumulation of the 3 x 2 k_chunk real products of one K chunk (the
      chunks are added in FP64): the probabilistic bound of Higham and Mary
      (SIAM J. Sci. Comput. 41, A2815 (2019)), lambda sqrt(n) u relative to the
      sum of magnitudes, with lambda = 8 (it fails with probability below
      2 n exp(-lambda^2 / 2) ~ 1e-13 n).  The worst-case n u bound is useless
      at K chunks of 10^5 values.
    """
    return 3 * 2.0 ** -16 + 8 * math.sqrt(6 * k_chunk) * U32


def fp32_chain_bound(n, m):
    """FP32 Chebyshev chains L_n and R_m against FP64 ones, relative to B_nm.

    A step v_{k+1} = 2 H~ v_k - v_{k-1} rounds each element of the new vector
    once per term (Z neighbours, the on-site term, the w term: <= 6 terms on
    these lattices), an error <= 6 u |terms|.  A rounding error made at step j
    reaches step n through U_{n-j}(H~) (Chebyshev polynomial of the second
    kind), whose size on [-1, 1] is <= n - j + 1, so the worst case grows
    quadratically; rounding errors of independent sign add up in quadrature,
    giving ~ n^1.5 for a random walk of them.  The test gates at
    (n + m + 2)^1.5 * 6 u * lambda / sqrt(3), lambda = 8 (the same confidence
    level as above), for the two chains of Gamma_nm.
    """
    return (n + m + 2) ** 1.5 * 6 * U32 * 8 / math.sqrt(3)


def fp32_moment_bound(n, n_active: int):
    """Gate for FP32-recursion moments against FP64 ones (the FP32 path has no
    exact pin; this is its stated accuracy).

    The FP32 error of mu_n has a part that averages over the orbitals
    (independent roundings of each step, of the start phases and of the
    on-site potentials: ~ 1/sqrt(n_active)) and a small coherent part (the
    hopping ratio t/de- rounded once).  Measured on the headline workload
    (graphene 4096^2, 2^25 orbitals, all 2048 moments of 32 vectors): 4e-8.
    Stated accuracy there: 1e-6 for every moment; smaller lattices get
    1e-6 * sqrt(2^25 / n_active), the averaging part's scaling.
    """
    import numpy as np
    tol = 1e-6 * math.sqrt(max(1.0, 2.0 ** 25 / n_active))
    return np.full(np.shape(n), tol) if np.ndim(n) else tol

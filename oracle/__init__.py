"""CPU FP64 oracle for the KPM hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the HIP path
computes, written from the paper (KITE, arXiv:1910.05194):

* ``rng``     counter-based SplitMix64 streams (published definition).
* ``lattice`` explicit sparse (CSR) Hamiltonians built bond by bond
              (Sec. 3(a) pattern rules, Sec. 3(d) honeycomb listing, eq. HQAHE
              Rashba term, Sec. 4 Peierls substitution), Anderson disorder and
              vacancies.
* ``kpm``     rescaling (eqs. rescalingH / rescalingE), the matrix Chebyshev
              recursion (eq. e6), stochastic-trace moments computed directly
              as <r|T_n(H)|r> (Sec. 2(c)), the Jackson kernel and the DOS
              reconstruction (eqs. e7, delta_function_cheb_expansion).
* ``cond``    velocity operators [r^a, H] and [r^a, [r^b, H]] (eq. generalized
              velocity), the rank-2 and rank-1 Gamma tensors (eq. Gammanm) by
              plain inner products, the T = 0 longitudinal conductivity from
              Gamma, the Kubo-Bastin DC and optical conductivities with the
              Fermi function (eqs. cond 1st order, conductivity_1st_order), the
              single-shot conductivity, and eigenstate / k-space references.
* ``evolve``  wave-packet time evolution: the Chebyshev-Bessel expansion of
              exp(-i H dt / hbar) (Sec. 4), the Gaussian packet and its spin
              and position observables.
* ``mlp``     FP64 forward/backward/Adam of the moment-extrapolation MLP.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(the product package never imports it) and uses no GPU.  Functions whose
result is not tied to something fixed outside this code say "parity
unpinned" in their docstring.
"""

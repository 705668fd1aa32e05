"""Plain, slow, double-precision CPU oracle for the many-variable VMC hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it.  The GPU library
never calls it, never links it and shares no code with it: it exists to say
what the right answer is.

Everything here computes the plain definitions of the paper (arXiv:1711.11418,
"mVMC -- open-source software for many-variable variational Monte Carlo
method"), not the fast algorithms the GPU uses:

* philox.py       -- Philox4x32-10 counter-based generator (Salmon et al.,
                     SC'11), the stand-in for the paper's Mersenne twister
                     (section 3.1.1); both sides implement it independently.
* pfaffian.py     -- Parlett-Reid Pfaffian with partial pivoting (the method
                     of the Pfaffian library the paper cites, section 3.2.1)
                     and a brute-force perfect-matching sum.
* wavefunction.py -- log <x|psi> from scratch: Pfaffian of X_IJ = F_IJ - F_JI
                     (section 3.2.1, Eqs. Pf and AP-Pf), Gutzwiller and
                     Jastrow factors (section 3.2.3), an RBM factor, and the
                     momentum / point-group projection sum_p w_p T_p of the
                     pair-product part (section 3.2.2).
* sampler.py      -- Metropolis chain with a full recomputation per proposal
                     (section 3.1, Eq. MC; hopping update of Fig. 5a).
* measure.py      -- local energy and O_k = d ln<x|psi>/d alpha_k
                     (section 3.3.1, Eq. DiffPf; appendix C).
* enumerate.py    -- exhaustive sums over all configurations of tiny lattices.
* ed.py           -- exact diagonalisation of the Hubbard Hamiltonian
                     (section 2.3, Eq. GHam with H_U).
* sr.py           -- SR overlap, force and update (section 3.3.1,
                     Eq. SR_equation_system), Cholesky solve and the CG method
                     of Algorithm 1 (section 3.3.2).
* lanczos.py      -- first-step power-Lanczos (section 3.4): F(x, H^2) by two
                     applications of H with every end point from scratch, the
                     four moments, E_1(alpha) and the optimal alpha_1.

Parity status: every function here is pinned by a test under tests/ that
checks it against closed forms, invariants or brute force (see the module
docstrings); nothing is "parity unpinned" except the variational gain of the
RBM factor, which is a comparison of energies and not a computed value.
"""

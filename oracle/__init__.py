"""FP64 CPU oracle for the HMC density sampler of Jasche & Wandelt (2013),
"Methods for Bayesian power spectrum inference with galaxy surveys".

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
It shares no code with the HIP library (``paper_1306_1821_amd``) and never
imports it; both sides receive their inputs from ``synth`` (seeded input
generators that hold none of the method's arithmetic).

Everything is plain numpy/scipy in float64, written to be checked by eye
against the paper:

* ``grid``    -- multi-index grid, DFT convention (Appendix "Discrete Fourier
                 transformation"), k-shells sigma_m / n_m (eq. INVERSE_GAMMA
                 and the shell sum that follows it).
* ``philox``  -- Philox4x32-10 counter-based generator (Salmon et al. 2011) and
                 Box-Muller normals: the method's own random numbers.
* ``model``   -- data model coefficients, Wiener potential psi and its force
                 (eqs. Wiener_Posterior_psi / Wiener_Posterior_force), the
                 Fourier-diagonal mass (eq. Mass_matrix and the text after it).
* ``hmc``     -- Hamiltonian, KDK leapfrog and Metropolis accept (Sec. "The HMC
                 algorithm", eqs. Hamiltonian, HAMILTON1_a/2_a, acceptance_rule).
* ``gibbs``   -- conditional draws: P(k) via chi^2 (eqs. XI_SQUARE, PS_sample),
                 Nbar via GIG (eq. GIG_post, Appendix A), bias via a normal
                 (Appendix B), and the block sweep (eq. multiblock).
* ``rj``      -- the joint (P, delta) move with the deterministic transition
                 (eq. det_trans; Appendix C, eq. spec_posterior_MIXING_1).

Readings of places where the paper is silent or inconsistent are listed in
the module docstrings where they are used.
"""

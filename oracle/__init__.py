"""Plain, slow FP64 CPU oracle for the HyperSARA primal-dual hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The HIP library in
``paper_1806_04596_amd`` never imports it and shares no code, headers, tables
or constant generators with it.

Every function follows a passage of Abdulaziz, Dabbech & Wiaux, "Wideband
super-resolution imaging in radio interferometry via low rankness and joint
average sparsity models (HyperSARA)", MNRAS (arXiv:1806.04596), cited by
section, equation label or algorithm step.  Where the paper is silent the
reading taken is stated in the docstring.

Modules
-------
nufft    : measurement operator Phi = Theta G F Z and its adjoint (Sec. 2.1)
wavelets : SARA dictionary Psi (Dirac + Daubechies db1..db8) (Sec. 2.3)
prox     : proximity operators and dual updates (Sec. 3.3, eq:md)
precond  : sampling-density preconditioner U (Sec. 3.3)
binning  : definition of the visibility tile/region order (host logic)
pd       : one adaptive-PPD iteration (Algorithm 2), step sizes, reweighting
           (Algorithm 1), power iteration, mu estimate.

Parity status of each function is stated in its docstring; all functions
are pinned by tests in ``tests/test_oracle_*.py``.
"""

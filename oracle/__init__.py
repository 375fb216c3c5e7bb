"""Plain FP64 CPU oracle for the higher-order lattice-kinetic Poisson scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library under
``paper_1504_05869_amd/`` and its Python binding) imports, links or runs any
file here.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.

It is written from the paper (Mendoza, Succi, Herrmann, "High-Order Kinetic
Relaxation Schemes as High-Accuracy Poisson Solvers"), slow and obviously
correct, and shares no code, header, table or constant generator with the GPU
path:

* ``lattice``  -- velocity sets, quadrature weights and sound speeds solved
  from the orthogonality condition (Eq. quadrature / Eq. quad3, Appendix), and
  the Hermite-designed equilibrium and source shapes phi_i, chi_i
  (Eqs. omega:eq, chi:eq, omega:eq3, chi:eq3).
* ``exact``    -- the discrete moment identities of Sec. 4 checked in exact
  (rational / algebraic) arithmetic.
* ``sweep``    -- the discrete BGK iteration (stream, moment, collide + source)
  in plain C (``sweep.c``) and as a numpy ``roll`` reference.
* ``spectral`` -- the exact fixed point of that iteration on a periodic grid,
  one Fourier mode at a time.
* ``dense``    -- the same fixed point by a dense linear solve on tiny grids.
* ``bf16dev``  -- the same sweep with the post-collision state stored as an
  FP32 moment and BF16 deviations (storage-precision ablation).
* ``generator`` -- the search for new velocity sets from the quadrature
  conditions (Sec. 4), with positive weights and a von Neumann stability
  filter.
* ``drift``    -- the advection-diffusion variant (the equilibrium of a
  Gaussian moved by a uniform drift) and its exact complex fixed point.

Every function with no independent pin says "parity unpinned" in its
docstring; at present there is none.
"""

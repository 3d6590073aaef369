"""FP64 CPU oracle of the stratified Taylor-Green DDF lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the HIP library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it; the product library (``paper_2605_14505_amd``) never does, and it shares no
code, tables or helpers with it.

Modules:
  lattice  Table 1 velocity sets in exact rationals
  model    the vectorised FP64 step, set-up and diagnostics (Section 2, Eqs. (5)-(26))
  micro    a node-by-node pure-Python transcription of the same step
  linear   the linearised lattice propagator (exact shear-mode decay per step)
  mlp      FP64 forward/backward of the per-node correction network

Every function here is pinned by the CPU tests (``pytest -m "not gpu"``) to
something other than itself: Table 1 as printed, exact isotropy identities,
conservation, closed forms at t = 0, the linear decay and internal-wave
theory, and finite differences.
"""

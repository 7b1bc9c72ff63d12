"""FP64 CPU oracle for the fictitious-wave-domain CSEM FDTD hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the package-level smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP path: its finite-
difference weights come from Fornberg's recursion (the HIP host side solves
the Vandermonde system with the Bjorck-Pereyra algorithm), and its time
stepper is a separate plain-C file with no tiling or fusion.

What it computes, step by step, in the paper's order (Algorithm 1):
  setup      padded coordinates, FD tables, dt, CPML tables, wavelet,
             interpolation weights (Sections 3.1, 3.2, 3.4, 3.5)
  per step   curl H (+CPML) -> inject J -> update E -> record (DFT)
             -> curl E (+CPML) -> update H                        (Section 3.1)
  after      Green's-function normalisation                        (Section 2.2)

Pins (tests/test_oracle_*.py): uniform-grid closed-form coefficients,
polynomial exactness on non-uniform grids, the plane-wave symbol of the
staggered derivative (appendix on dispersion), the CFL closed form, the
analytic whole-space electric dipole (also on a strongly stretched z axis,
which pins the injection control volume and the padding), the z-domain
identity solved by a sparse direct solver, reciprocity (also on the marine
stretched axis with CPML), omega0- and wavelet-invariance, CPML reflection;
the discrete adjoint by central differences of the forward; the air
boundary's ghost fills by exact harmonic and potential fields and by the
z-domain solve with the fills as operators; the convergence stop.
Layered and blocky models are pinned as discrete operators (the z-domain
identity holds for any model); their discretisation error against the
continuous layered-earth solution is not measured (no layered-earth solver
is available), and it is not a parity matter: both implementations
discretise identically.
"""

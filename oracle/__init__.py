"""FP64 CPU oracle for the decoupled phase-field scheme of Yang, Christov & Dong,
"Phase Field Modeling and Numerical Algorithm for Two-Phase Dielectric Fluid Flows"
(arXiv 2305.09020).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code, table or helper with the HIP library
under ``paper_2305_09020_amd/``.

What it computes: the fully discrete scheme of Sec. 3 -- Algorithm 1 (2D, C0
spectral elements, Sec. 3.2.1) and Algorithm 2 (3D, Fourier x spectral elements,
Sec. 3.2.2) -- written out plainly:

* assembled SciPy sparse matrices (mass, stiffness, element-local gradient
  operators) built by looping over elements,
* SciPy sparse LU of each constant-coefficient system (Dirichlet rows
  eliminated), with no static condensation, no fast diagonalisation, no
  sum factorisation and no mixed precision,
* numpy FFTs along the homogeneous z direction (3D).

Modules:
  sem          -- GLL rule, Lagrange differentiation matrix, tensor mesh, sparse
                  element operators (Sec. 3.2.1 function spaces).
  scheme       -- parameters and derived constants (Sec. 3.1), the 2D and 3D
                  time steps (eqs. 54-59 and 74-78), the initial-potential
                  iteration (Remark 3.1), the equilibrium marching (eqs. 15-16).
  manufactured -- symbolic source terms for the manufactured solutions of
                  Sec. 4.1 (eqs. 80, 81).
"""

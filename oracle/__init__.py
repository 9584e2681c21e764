"""Plain FP64 CPU oracle for the EBIT phase-change elliptic path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(it reads the seeded inputs from ``ebit_inputs`` like the GPU side does).

The oracle computes, step by step and with no blocking or fusion, the
discrete problem the paper (Long, Pan & Zaleski, "A Front-Tracking
approach for phase change: the EBIT method") defines on a uniform grid:

  geometry.py  EBIT markers -> per-cell interface facet -> cut fraction theta
               per link, cell flags                     (Sec. 2.1, Sec. 2.4)
  heat.py      implicit per-phase diffusion with T = T_sat imposed sharply
               at theta (Eqs. energy_diffusion, ghost_T, Txx_ghost)
  flux.py      one-layer ghost fill from Eq. ghost_T and the mass flux from
               one-sided normal gradients (Eqs. mass_flux_computation,
               normal_gradient)
  project.py   ghost velocities from the mass-flux jump (Eq. ghost_velocity),
               the variable-density Poisson problem (Eqs. Poisson_equation,
               poisson_ghost_fluid) and the face-velocity update
  solve.py     sparse direct solve (SciPy SuperLU) of the assembled systems
  mg.py, mg.c  plain FP64 geometric multigrid (Galerkin aggregation, PCG,
               long-double refinement) for grids too large to factor
  extend.py    narrow-band extension of a cell field across the interface by
               pseudo-time upwind transport (Eq. extrapolation)
  onefluid.py  one-fluid projection: one face velocity field and the
               phase-change source in the interface cells (Eq. pc_source)
  advect.py    interfacial velocity at cell centres (Eq. jump_interfacial_vel)
               and at markers (bilinear), EBIT marker motion in 1D passes
               with the circle-fit re-intersection (Sec. 2.1, 2D)
  energy.py    the advection step of the energy equation: explicit Euler
               with third-order WENO derivatives, per phase (Eq.
               energy_advection)
  volume.py    liquid volume fraction of each cell from the EBIT segments
               (2D, Sec. 2.2 and Sec. 3.1)
  closed.py    closed forms used as pins (Stefan problem, Sec. 3.1)

Parity unpinned: the 3D facet rule beyond planar exactness (the paper's EBIT
is 2D only) and saddle cells.  Every other function is pinned by tests under
tests/ (the first-order fallback of the mass-flux stencil by a thin slab
worked out by hand).
"""
from . import geometry, heat, flux, project, solve, closed, pipeline, extend, onefluid, mg, advect, energy, volume  # noqa: F401
from .geometry import GeometryError  # noqa: F401

"""CPU FP64 oracle for the SiPO PDHG hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct NumPy/SciPy implementation of
what the HIP path computes, written from the paper (Woo, Lee, Taylor,
"Scale-invariant projection optimization in tomographic volumetric additive
manufacturing"):

  * ``geometry``  -- object grid, detector, angles, vial (Sec. 2.2, Fig. 2)
  * ``projector`` -- explicit sparse backprojector P^T and its transpose P,
                     with Beer-Lambert attenuation (Eq. 2-3)
  * ``blur``      -- the object-space PSF operator K (Eq. 3, Sec. 3 set-up)
  * ``regions``   -- gel / band / exterior partition and active rays (Fig. 2)
  * ``lp``        -- the Charnes-Cooper LP in its general, Case-1 and Case-2
                     forms (Eq. 19-24, 32-37, 40-45), assembled explicitly and
                     solved with HiGHS
  * ``simplex``   -- a dense two-phase simplex for tiny instances
  * ``kkt``       -- KKT residuals (Supp. 6.1, Eq. 47-51) and Farkas checks
  * ``pdhg``      -- plain and restarted PDHG (Sec. 2.8) in FP64
  * ``metrics``   -- DTVR, DSR, PSR (Eq. 6-8, 46), post-scaling (Eq. 25-28)

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code with the HIP path; the only common module
is ``sipo_inputs`` (seeded input generators, none of the method's arithmetic).
Functions with no independent pin say "parity unpinned" in their docstring.
"""

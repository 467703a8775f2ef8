"""Oracle for the phonon D2Q8 lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the product package never imports it
and shares no code with it.

* ``ref``          -- ctypes front end of the plain FP64 C time-stepper.
* ``bloch``        -- exact solution on periodic grids, one 8x8 matrix power per
                      Fourier mode (independent of the time-stepper).
* ``closed_forms`` -- the paper's analytic results (Eqs. 52, 61-62, 68-71) and
                      the parameter mapping (Eqs. 48-49).
"""

"""Oracle for the phonon lattice Boltzmann hot path (D2Q8, and D3Q14 in 3D).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the product package never imports it
and shares no code with it.

* ``ref``          -- ctypes front end of the plain FP64 C time-stepper.
* ``bloch``        -- exact solution on periodic grids, one 8x8 matrix power per
                      Fourier mode (independent of the time-stepper).
* ``ref.Oracle3D`` -- the FP64 C time-stepper of the D3Q14 lattice
                      (``phonon_oracle_d3q14.c``; weights derived from the
                      moment identities of Sec. 2.3).
* ``bloch_d3q14``  -- exact periodic D3Q14 solution, 14x14 matrix power per
                      mode, with the weights solved from those identities.
* ``closed_forms`` -- the paper's analytic results (Eqs. 52, 61-62, 68-71) and
                      the parameter mapping (Eqs. 48-49).
"""

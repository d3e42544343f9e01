"""Reference ("oracle") implementations used to check the HIP path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this package.
The product library never imports it and shares no code with it.

Contents
--------
lbm_oracle.c    plain FP64 C implementation of the two-component D2Q9 step
lbm.py          ctypes wrapper and whole-run helpers around it
lbm3d_oracle.c  the same step on the D3Q19 lattice (tubes, periodic boxes)
lbm3d.py        ctypes wrapper around it
young_laplace.py quasi-static Young-Laplace critical pressure (planar, axisymmetric)
analysis.py     tanh / circle / Laplace fits and the Bond number (Eqs. 11-18)
driver.py       critical-pressure bisection on top of the oracle step
mlp.py          FP64 multilayer perceptron (forward, backward, Adam)
"""

"""MI355X-native split-step SSA for stochastic metapopulation disease spread
(the method of SimInf, arXiv 1605.01421).

Submodules:

* ``siminf`` -- ctypes binding of the C-ABI library ``libsiminf.so`` (HIP,
  gfx950): model creation, runs, batches, trajectories, prevalence
  reduction and the surrogate MLP kernels.
* ``workloads`` -- seeded synthetic inputs (no method arithmetic).
* ``surrogate`` -- training / inference driver for the learned surrogate.

Importing the package loads nothing; ``siminf`` loads the HIP library on
first use and raises if it is missing.
"""

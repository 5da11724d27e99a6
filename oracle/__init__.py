"""Plain FP64 CPU oracle of the MOND particle-mesh step.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
of the package entry file and the ``cpu_baseline`` leg of the benchmark may
import or run anything in this package.  The HIP library never calls it and
shares no code with it: the only common module is the seeded input generator
package ``workloads``, which holds none of the method's arithmetic.

Modules
-------
pm       deposit, Newton solve, AQUAL fixed-point iteration, smoothed force,
         leapfrog and diagnostics, in the order of the paper's flow scheme
         (appendix "Flow scheme of the PM code").
linearised
         the step-to-step increments of the fields with the linearised
         algebraic equations and FP16 storage (Sect. 5, item (v)); no kernel
         implements it yet.
convnet  FP64 3D conv encoder-decoder (forward, backward, Adam) for the learned
         starting guess.  Parity unpinned against the paper (the paper has no
         such network); pinned by finite differences and closed forms.
"""

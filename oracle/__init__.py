"""Plain FP64 CPU oracle for the non-orthogonal MRT lattice Boltzmann update with the
pseudopotential multiphase model of Fei et al., "Modeling realistic multiphase flows using
a non-orthogonal multiple-relaxation-time lattice Boltzmann method" (arXiv 2306.16274).

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously-correct reference that the
GPU path is checked against. Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product library never does, and it shares no code,
tables or constants with the HIP path.

Everything is numpy float64. Matrix-vector products use the dense transformation matrix M
and its exact rational inverse; the formulas follow the paper's order and notation:

* ``lattice``     velocity sets, weights, moment set, M, M^-1, S, m^eq, F~   (Sec. II A-B, App. C)
* ``eos``         piecewise-linear and Carnahan-Starling pressure, square-root psi,
                  Maxwell coexistence densities                              (Sec. II C, Sec. III A)
* ``lbm``         forces, collision in moment space, streaming with halfway bounce-back,
                  initial state, macroscopic moments, totals and the liquid
                  diagnostics (liquid nodes per plane, in contact, volume)     (Sec. II, App. B, Sec. III E, IV)
* ``splitmix``    SplitMix64 counter generator for the interface noise of the initial state
"""

"""MI355X-native hot path of the Eulerian phase-field FSI method
(Mao & Jaiman, arXiv 2402.10348): one partitioned nonlinear iteration of a
time step behind the C ABI in include/eft.h.

Importing the package loads nothing; ``paper_2402_10348_amd.eft`` binds the
HIP library and raises if it is missing.
"""

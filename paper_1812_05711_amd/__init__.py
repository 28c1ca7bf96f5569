"""MI355X-native (gfx950, HIP) coupled TRT lattice Boltzmann / FFT-Poisson
electroconvection time step.  The compute path is the HIP library
liblbm_ec.so (C ABI in include/lbm_ec.h); lbm_ec.py binds it."""

"""HMC density sampler of Jasche & Wandelt (2013) on AMD MI355X (gfx950).

The compute path is libhmc.so (HIP kernels behind the C-ABI of include/hmc.h);
``binding`` marshals arguments to it from Python, ``diagnostics`` holds the
chain statistics (ESS, split R-hat, autocorrelation length, burn-in xi).
"""

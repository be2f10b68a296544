"""MI355X (gfx950) ADMM reconstruction for convolutional inverse problems.

The compute path is the HIP library ``libcip.so`` (C ABI in include/cip.h);
``paper_2006_08303_amd.cip`` is a thin ctypes binding that marshals torch
device tensors to it. ``synth`` holds the seeded synthetic input generators.
"""

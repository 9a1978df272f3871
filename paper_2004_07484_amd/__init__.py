"""MI355X (gfx950) sphere renderer of Pulsar: HIP kernels behind a C ABI.

Import ``paper_2004_07484_amd.renderer`` for the PyTorch front end and
``paper_2004_07484_amd._capi`` for the raw binding of include/pulsar.h.
"""

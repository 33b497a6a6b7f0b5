"""MI355X-native DAMAS on a wavelet-compressed computational grid.

``paper_1608_05179_amd.damas`` is the thin ctypes binding of the HIP
library (``libdamas_hip.so``); ``paper_1608_05179_amd.synth`` builds seeded
synthetic workloads.  Importing the package loads neither.
"""
__all__ = ["damas", "synth", "build"]

"""MI355X-native thin-disc kinematic model evaluation (Bekiaris et al. 2016).

Submodules are imported explicitly: ``inputs`` (seeded synthetic workloads),
``gbk`` (ctypes binding of the HIP library libgbk.so).
"""

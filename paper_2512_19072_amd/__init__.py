"""MI355X (gfx950) implementation of Fast Optimal Transport (FOT) for holographic beam
shaping (arXiv 2512.19072): the HIP library libfot.so behind include/fot.h, its ctypes
binding (:mod:`.fot`), and seeded synthetic workloads (:mod:`.workloads`)."""
__version__ = "0.1.0"

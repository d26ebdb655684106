"""MI355X-native operators and eigensolver of the mixed-basis (2D plane waves x
B-splines) Kohn-Sham method: HIP kernels behind a C ABI (libmbks.so), with a thin
ctypes binding in ``mbks`` and seeded synthetic problems in ``workloads``."""

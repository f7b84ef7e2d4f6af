"""MI355X-native shift-and-invert solver for damped-wave QEPs discretised with
IGA / refined IGA (arXiv 2112.14064).  The compute path is libriga.so (HIP for
gfx950); `riga` is its ctypes binding and `workloads` the seeded inputs."""

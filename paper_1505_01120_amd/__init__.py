"""SparkCL (arXiv:1505.01120) map -> reduce offload hot path, MI355X-native.

MapCL, MapCLPartition and ReduceCL (paper sec. 3.1.3) over a registry of three
built-in partition kernels, as hand-written HIP for gfx950 behind a C ABI
(include/sparkcl.h).  This package is the ctypes binding of that library.
"""
from .sparkcl import *  # noqa: F401,F403
from .sparkcl import Context, Result, Task, TaskArray, Tuning, load, task, task_array  # noqa: F401

"""MI355X-native DG S_N sweep + Second Moment Method (libsmm) and its Python
binding.  See include/smm.h for the C ABI."""
from .smm import *  # noqa: F401,F403
from .workload_io import problem_from_workload  # noqa: F401

"""MI355X-native element derivatives, BSR assembly and Newton steps (SymX hot path).

Native code lives in csrc/ (HIP kernels, the C-ABI declared in include/symx.h
and the build-time symbolic generator); symx.py is the ctypes binding.
"""

"""MI355X-native pseudospectral P_N radiative-transport stepper.

The compute path is the HIP library ``librte.so`` (C-ABI in include/rte.h);
``paper_1801_06364_amd.rte`` is its ctypes binding.
"""

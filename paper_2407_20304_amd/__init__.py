"""MI355X-native joint object-and-probe holotomography gradient.

The compute path is the HIP library `libholo.so` (C ABI in include/holo.h);
`paper_2407_20304_amd.holo` is its thin Python binding.
"""

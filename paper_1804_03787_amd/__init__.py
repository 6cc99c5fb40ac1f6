"""MI355X-native hot path of multi-scale generalized plane match (arXiv 1804.03787).

The compute path is the HIP library ``libmsgpm.so`` (C-ABI declared in
include/msgpm.h); ``paper_1804_03787_amd.msgpm`` is its thin Python binding.
``paper_1804_03787_amd.synth`` generates seeded synthetic frame pairs.
"""

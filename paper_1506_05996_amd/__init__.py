"""MI355X (gfx950) spectral-element Poisson solver: C-ABI HIP library + binding.

``paper_1506_05996_amd.sem`` loads ``libsem.so`` (built in-tree by
``paper_1506_05996_amd.build``) and fails loudly when it is missing.
"""

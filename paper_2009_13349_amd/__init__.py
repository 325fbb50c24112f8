"""MI355X-native inclusion-based continuous collision detection (CCD).

The root finder of Wang et al. 2021 (Algorithm 2, with the minimum-separation
variant of Sec. 6) runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/ccd.h``; `paper_2009_13349_amd.ccd` is the thin Python
binding over it.  `paper_2009_13349_amd.workloads` generates seeded synthetic
query sets.
"""

"""MI355X (gfx950) Haar-tSVD denoiser: HIP kernels behind the C ABI of
include/hts.h, with a thin torch binding (paper_2508_10307_amd.api) and
seeded synthetic workloads (paper_2508_10307_amd.synth).  The shared
library is loaded on first use."""

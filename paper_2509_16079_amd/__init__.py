"""MI355X-native rollout engine for the vortex-particle glider planner of
Gupta et al., arXiv 2509.16079.

The compute path is the C-ABI library ``libvpm.so`` (hand-written HIP for
gfx950) declared in ``include/vpm.h``; :mod:`paper_2509_16079_amd.vpm` is its
thin Python binding and :mod:`paper_2509_16079_amd.workloads` draws seeded
synthetic inputs.
"""

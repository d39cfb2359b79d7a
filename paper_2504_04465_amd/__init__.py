"""MI355X-native refined-grid lattice Boltzmann hot path (arXiv 2504.04465).

The compute path is the HIP library ``liblbm.so`` behind the C-ABI declared in
``include/lbm.h``; :mod:`paper_2504_04465_amd.lbm` is its thin Python binding
and :mod:`paper_2504_04465_amd.workloads` describes the synthetic inputs.
"""
__all__ = ["lbm", "workloads"]

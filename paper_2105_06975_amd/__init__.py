"""MI355X-native saddle-point solver for weak-constraint 4D-Var (Tabeart & Pearson).

The compute path is the HIP library ``libsvar.so`` (C ABI declared in include/svar.h);
``paper_2105_06975_amd.svar`` is its thin ctypes binding.  ``workloads`` draws the
seeded synthetic inputs.  Submodules are imported lazily so that the input generators
work on machines without the built library.
"""
__all__ = ["svar", "workloads"]

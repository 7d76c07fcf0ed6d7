"""MI355X-native Friedkin-Johnsen equilibrium and opinion indices.

    from paper_2101_08143_amd import fj          # ctypes binding of libfjgpu (include/fj.h)
    from paper_2101_08143_amd import workloads   # seeded synthetic graphs and opinions

The HIP library is built in-tree by `python -m paper_2101_08143_amd.build`.
"""
__all__ = ["fj", "workloads"]

"""MI355X-native hot path of Dynamic Ray Tracing (arXiv 2205.00237).

    from paper_2205_00237_amd import scenes          # seeded synthetic workloads (numpy only)
    from paper_2205_00237_amd.drt import Context     # the HIP library through its C ABI

`drt` loads the in-tree libdrt.so (built by paper_2205_00237_amd.build) and raises if it is
missing: there is no CPU or PyTorch fallback.
"""
__all__ = ["scenes", "drt", "build"]

"""ipx: FP64 unbinned-likelihood engine for AMD MI355X (gfx950).

    from paper_1706_01420_amd import ipx      # ctypes binding of libipx.so
    python -m paper_1706_01420_amd.build      # compile libipx.so in-tree

The binding is imported explicitly (it loads the HIP runtime and the library).
"""
__all__ = ["ipx", "workloads", "build"]

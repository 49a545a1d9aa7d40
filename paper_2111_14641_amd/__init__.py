"""MI355X (gfx950) randomized block Gram-Schmidt QR.

The computation lives in the HIP library librbgs.so (C ABI: include/rbgs.h);
`binding` is a thin ctypes layer over it that takes PyTorch CUDA tensors for
memory and streams.  `workloads` builds the seeded synthetic input matrices.
"""
__all__ = ["binding", "workloads"]

"""Ternary (EVP) quantised embedding search on AMD MI355X (gfx950).

The compute path is the HIP library libtq.so (C ABI in include/tq.h); the
Python binding in `tq` only marshals torch tensors to it.
"""

"""TFHE gate bootstrapping and CMUX memory on AMD Instinct MI355X (gfx950).

``_native`` is the ctypes binding of libvsp (the C ABI in include/vsp.h); ``device`` wraps
it with torch tensors for device memory and streams; ``client`` is the key owner's side
(key generation, encryption, decryption) in numpy.
"""
from . import client  # noqa: F401
from ._native import (AND, ANDNOT, NAND, NOR, NOT, OR, ORNOT, VSP_BATCHED, VSP_PER_GATE, XNOR, XOR,  # noqa: F401
                      VspError)

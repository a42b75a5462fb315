"""Hash of the kernel sources and of the host code that sets their launch
order, stored with every measured traffic figure so that a figure taken on
other kernels or another launch order is never reported as current."""
import hashlib
import os

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/kernels.hip", "csrc/lbm_cell.h", "csrc/hlbm_internal.h", "csrc/api.cpp"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(PKG, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

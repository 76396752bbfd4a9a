"""ctypes binding of libhoqri_gather.so (include/hoqri_gather.h), the
gather-only pass (the factor-row gathers of a TTMcTC pass and nothing else),
and the index streams it is run on.

A mode's stream is what that mode's pass gathers, in the plan's order: the
slices of mode n in index order, inside each slice the nonzeros ordered by
the degree labels of the other modes (ascending modes, C order; labels by
descending slice size, ties by index), and per nonzero the label of each
other mode, which is the row the pass reads from that mode's factor kept in
label order.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhoqri_gather.so")
_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run paper_2510_16930_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.hoqri_gather_only.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                                                 ctypes.c_int32, ctypes.c_void_p]
        L.hoqri_gather_only.restype = ctypes.c_int
        _lib = L
    return _lib


def check_operands(U1, U2, i1, i2, out, grid: int) -> None:
    """Host-side checks of gather_only's operands (the row-number range check
    runs two reductions on the device and synchronises: keep it out of a timed
    region). Raises ValueError."""
    import torch
    if U1.dtype != torch.float32 or U2.dtype != torch.float32 or U1.shape[1] != 16 or U2.shape[1] != 16:
        raise ValueError("tables must be float32 with 16 columns (64-byte rows)")
    if not (U1.is_contiguous() and U2.is_contiguous() and i1.is_contiguous() and i2.is_contiguous()):
        raise ValueError("operands must be contiguous")
    if i1.dtype != torch.int32 or i2.dtype != torch.int32 or i1.numel() != i2.numel() or i1.numel() % 16:
        raise ValueError("index streams must be int32 of one length, a multiple of 16")
    for i, U in ((i1, U1), (i2, U2)):
        if i.numel() and (int(i.min()) < 0 or int(i.max()) >= U.shape[0]):
            raise ValueError("index out of the table's rows")
    if out.dtype != torch.float32 or out.numel() < grid * 256:
        raise ValueError("out must hold grid*256 float32")


def gather_only(U1, U2, i1, i2, wide: bool, out, grid: int, stream=None, checked: bool = False) -> None:
    """One launch of hoqri_gather_only on `stream` (torch's current stream by
    default). U1, U2: float32 device tensors of 16 columns; i1, i2: int32
    device tensors of equal length, a multiple of 16, with values below the
    row counts of U1 and U2; out: float32 device tensor of grid*256 entries.
    The operands are checked first (check_operands) unless `checked` says the
    caller has done so for these same tensors."""
    import torch
    if not checked:
        check_operands(U1, U2, i1, i2, out, grid)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = load().hoqri_gather_only(U1.data_ptr(), U2.data_ptr(), i1.data_ptr(), i2.data_ptr(), i1.numel(),
                                  1 if wide else 0, out.data_ptr(), grid, ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hoqri_gather_only returned {rc}")


def degree_labels(idx, dims):
    """Per mode, the label of each nonzero's index: slices ordered by
    descending size, ties by index (int64 device tensors)."""
    import torch
    labs = []
    for m, d in enumerate(dims):
        deg = torch.bincount(idx[m].long(), minlength=d)
        order = torch.sort(-deg, stable=True).indices
        lab = torch.empty(d, dtype=torch.int64, device=idx.device)
        lab[order] = torch.arange(d, device=idx.device)
        labs.append(lab[idx[m].long()])
    return labs


def mode_stream(idx, labs, dims, n):
    """The two other modes' rows (int32 label streams) in mode n's pass order,
    and those two modes; 3-way tensors (idx: the coordinates, labs: from
    degree_labels)."""
    import torch
    if len(dims) != 3:
        raise ValueError("the gather-only pass covers 3-way tensors")
    o = [m for m in range(3) if m != n]
    key = idx[n].long() * (dims[o[0]] * dims[o[1]]) + labs[o[0]] * dims[o[1]] + labs[o[1]]
    perm = torch.sort(key).indices
    return labs[o[0]][perm].to(torch.int32).contiguous(), labs[o[1]][perm].to(torch.int32).contiguous(), o

"""ctypes binding of the hand-derived anisotropic-medium kernels
(include/raygraph_hand.h): the comparison baseline for the compiled path."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import raygraph as rgb  # loads torch's HIP runtime first

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraygraph_hand.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2508_15967_amd.build`")
_lib = C.CDLL(LIB_PATH)
_lib.rg_hand_last_error.restype = C.c_char_p
_lib.rg_hand_aniso_trace.restype = C.c_int32
_lib.rg_hand_aniso_adjoint.restype = C.c_int32
_lib.rg_hand_aniso_adjoint_workspace_size.restype = C.c_int32
MAXB = 32


class HandAniso(C.Structure):
    _fields_ = [("nb", C.c_int32), ("c", (C.c_double * 3) * MAXB), ("inv_w2", C.c_double * MAXB),
                ("m", (C.c_double * 6) * MAXB)]


def medium_struct(med) -> HandAniso:
    h = HandAniso()
    nb = len(med.scales)
    h.nb = nb
    for b in range(nb):
        for i in range(3):
            h.c[b][i] = float(med.centers[b][i])
        h.inv_w2[b] = 1.0 / float(med.widths[b]) ** 2
        for i in range(6):
            h.m[b][i] = float(med.mats[b][i])
    return h


def _p(t):
    return None if t is None else C.c_void_p(int(t.data_ptr()))


def _chk(st, where):
    if st != 0:
        raise RuntimeError(f"{where} failed ({st}): {_lib.rg_hand_last_error().decode()}")


def trace(hm, x0, k0, omega, s, dt, n_steps, x_out, k_out, ckpt_every=0, ckpt=None, block=0, stream=None):
    _chk(_lib.rg_hand_aniso_trace(C.byref(hm), C.c_uint32(x0.shape[-1]), _p(x0), _p(k0), _p(omega), _p(s),
                                  C.c_double(dt), C.c_int32(n_steps), _p(x_out), _p(k_out),
                                  C.c_int32(ckpt_every), _p(ckpt), C.c_int32(block),
                                  C.c_void_p(rgb._stream_handle(stream))), "rg_hand_aniso_trace")


def workspace_size(n, ckpt_every, block=0) -> int:
    b = C.c_size_t()
    _chk(_lib.rg_hand_aniso_adjoint_workspace_size(C.c_uint32(n), C.c_int32(ckpt_every), C.c_int32(block),
                                                   C.byref(b)), "rg_hand_aniso_adjoint_workspace_size")
    return int(b.value)


def adjoint(hm, omega, s, dt, n_steps, ckpt_every, ckpt, lx, lk, gx0, gk0, gs, block=0, stream=None,
            workspace=None):
    """The workspace (a torch uint8 tensor of at least workspace_size bytes)
    is allocated here when not given."""
    import torch
    n = int(omega.shape[-1])
    if workspace is None:
        workspace = torch.empty(max(1, workspace_size(n, ckpt_every, block)), dtype=torch.uint8,
                                device=omega.device)
    _chk(_lib.rg_hand_aniso_adjoint(C.byref(hm), C.c_uint32(n), _p(omega), _p(s),
                                    C.c_double(dt), C.c_int32(n_steps), C.c_int32(ckpt_every), _p(ckpt),
                                    _p(lx), _p(lk), _p(gx0), _p(gk0), _p(gs), C.c_int32(block),
                                    _p(workspace), C.c_size_t(workspace.numel()),
                                    C.c_void_p(rgb._stream_handle(stream))), "rg_hand_aniso_adjoint")

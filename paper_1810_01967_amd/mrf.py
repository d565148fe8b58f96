"""Thin ctypes binding of the C ABI in include/mrf.h.

Functions keep the C names (mrf_match, mrf_ipg_step, ...).  They only
marshal arguments: device buffers are torch CUDA tensors (torch is used for
device memory and the current stream), every step of the computation runs in
libmrf.so.  There is no fallback: a missing library or a failing call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrf.so")

MRF_OK = 0
MRF_E_INVAL, MRF_E_NOMEM, MRF_E_HIP, MRF_E_UNSUPPORTED, MRF_E_NUMERIC, MRF_E_NOCONV = -1, -2, -3, -4, -5, -6
MRF_STORE_BF16, MRF_STORE_FP8, MRF_BUILD_COVERTREE = 2, 4, 8
MRF_F64, MRF_F32 = 0, 1
MRF_EXHAUSTIVE, MRF_LEARNED, MRF_COVERTREE = 0, 1, 2
MRF_FP32, MRF_BF16, MRF_FP8, MRF_BF16X3 = 0, 1, 2, 3
MRF_VOXEL_MAJOR, MRF_FRAME_MAJOR = 0, 1
PRECISION = {"fp32": MRF_FP32, "bf16": MRF_BF16, "fp8": MRF_FP8, "bf16x3": MRF_BF16X3}

EXPORTS = ["mrf_last_error", "mrf_version", "mrf_dict_build", "mrf_dict_destroy", "mrf_dict_query",
           "mrf_dict_copy_atoms", "mrf_dict_compress", "mrf_dict_subspace", "mrf_dict_align", "mrf_dict_tree_info", "mrf_dict_tree_export", "mrf_match", "mrf_match_noalloc", "mrf_match_local", "mrf_net_create", "mrf_net_destroy",
           "mrf_net_size", "mrf_net_set_params", "mrf_net_get_params", "mrf_net_get_grads",
           "mrf_net_set_standardisation", "mrf_net_get_standardisation", "mrf_net_forward",
           "mrf_net_forward_bf16",
           "mrf_net_loss_grad", "mrf_net_adam", "mrf_net_noisy_batch", "mrf_net_train",
           "mrf_op_forward", "mrf_op_adjoint", "mrf_ipg_step", "mrf_ipg_solve", "mrf_quantize_rows",
           "mrf_nufft_create", "mrf_nufft_destroy"]


class MrfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mrf status {status}: {message}")
        self.status = status
        self.message = message


# --------------------------------------------------------------------------- structs
class DictDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("L", ctypes.c_int32), ("nparam", ctypes.c_int32),
                ("is_complex", ctypes.c_int32), ("atoms", ctypes.c_void_p),
                ("atoms_dtype", ctypes.c_int32), ("params", ctypes.c_void_p),
                ("grid_dims", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class DictInfo(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("L", ctypes.c_int32), ("nparam", ctypes.c_int32),
                ("is_complex", ctypes.c_int32), ("K", ctypes.c_int32), ("Kp", ctypes.c_int32),
                ("Kq", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("device_bytes", ctypes.c_int64), ("L_full", ctypes.c_int32), ("phase_aligned", ctypes.c_int32)]


class MatchOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("topk", ctypes.c_int32), ("atom_splits", ctypes.c_int32),
                ("net", ctypes.c_void_p), ("box_radius", ctypes.c_int32),
                ("fallback_corr", ctypes.c_float), ("recentre", ctypes.c_int32),
                ("eps", ctypes.c_float), ("tree_capacity", ctypes.c_int32),
                ("pd_phase", ctypes.c_void_p), ("no_certificate", ctypes.c_int32),
                ("certify_local", ctypes.c_int32)]


class MatchStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("zero_voxels", ctypes.c_int64),
                ("nonfinite", ctypes.c_int64), ("ms", ctypes.c_float),
                ("score_ms", ctypes.c_float), ("splits", ctypes.c_int32),
                ("fallbacks", ctypes.c_int64), ("recentred", ctypes.c_int64),
                ("local_atoms", ctypes.c_int64), ("proposal_ms", ctypes.c_float),
                ("fallback_ms", ctypes.c_float), ("search_ms", ctypes.c_float),
                ("distance_evals", ctypes.c_int64), ("tree_levels", ctypes.c_int32),
                ("first_box_atoms", ctypes.c_int64), ("cert_rescored", ctypes.c_int64),
                ("cert_rescanned", ctypes.c_int64), ("cert_scanned", ctypes.c_int64)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("unique_atoms", ctypes.c_int32), ("imax", ctypes.c_int32),
                ("entries", ctypes.c_int64), ("sigma", ctypes.c_double)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("batch", ctypes.c_int32), ("epochs", ctypes.c_int32),
                ("lr", ctypes.c_float), ("lr_min", ctypes.c_float), ("snr_lo", ctypes.c_float),
                ("snr_hi", ctypes.c_float), ("seed", ctypes.c_uint64)]


class TrainStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("first_loss", ctypes.c_double),
                ("last_loss", ctypes.c_double), ("ms", ctypes.c_float)]


class Op(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("L", ctypes.c_int32),
                ("nslices", ctypes.c_int32), ("nsamples", ctypes.c_int64),
                ("samp_off", ctypes.c_void_p), ("samp_idx", ctypes.c_void_p),
                ("dcf", ctypes.c_void_p), ("ncoils", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("smaps", ctypes.c_void_p), ("nufft", ctypes.c_void_p)]


class StepStats(ctypes.Structure):
    _fields_ = [("dx2", ctypes.c_double), ("adx2", ctypes.c_double), ("f_in", ctypes.c_double),
                ("f_out", ctypes.c_double), ("ms", ctypes.c_float), ("distance_evals", ctypes.c_int64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("mu0", ctypes.c_float), ("zeta", ctypes.c_float), ("adaptive", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("rel_tol", ctypes.c_double),
                ("max_shrinks", ctypes.c_int32), ("kappa", ctypes.c_int32),
                ("match", MatchOpts)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("total_shrinks", ctypes.c_int32),
                ("cap", ctypes.c_int32), ("f", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("shrinks", ctypes.c_void_p), ("f0", ctypes.c_double), ("ms", ctypes.c_float),
                ("fallbacks", ctypes.c_int64), ("distance_evals", ctypes.c_int64)]


_LIB = None


def lib():
    """Load libmrf.so (built in-tree by build.py); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1810_01967_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.mrf_last_error.restype = ctypes.c_char_p
        L.mrf_version.restype = ctypes.c_char_p
        for name in EXPORTS[2:]:
            getattr(L, name).restype = ctypes.c_int
        L.mrf_dict_build.argtypes = [ctypes.POINTER(DictDesc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.mrf_dict_destroy.argtypes = [ctypes.c_void_p]
        L.mrf_dict_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(DictInfo)]
        L.mrf_dict_copy_atoms.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        L.mrf_dict_compress.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]
        L.mrf_dict_subspace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.mrf_dict_align.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                     ctypes.POINTER(ctypes.c_void_p)]
        L.mrf_nufft_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.mrf_nufft_destroy.argtypes = [ctypes.c_void_p]
        L.mrf_match.argtypes = [ctypes.c_void_p, ctypes.POINTER(MatchOpts), ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.POINTER(MatchStats), ctypes.c_void_p]
        L.mrf_match_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(MatchOpts), ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
        L.mrf_dict_tree_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(TreeInfo)]
        L.mrf_dict_tree_export.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
        L.mrf_match_local.argtypes = [ctypes.c_void_p, ctypes.POINTER(MatchOpts), ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(MatchStats), ctypes.c_void_p]
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.mrf_net_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_void_p)]
        L.mrf_net_destroy.argtypes = [vp]
        L.mrf_net_size.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.mrf_net_set_params.argtypes = [vp, vp, i64]
        L.mrf_net_get_params.argtypes = [vp, vp, i64]
        L.mrf_net_get_grads.argtypes = [vp, vp, i64]
        L.mrf_net_set_standardisation.argtypes = [vp, vp, vp, vp]
        L.mrf_net_get_standardisation.argtypes = [vp, vp, vp, vp]
        L.mrf_net_forward.argtypes = [vp, vp, i64, vp, vp]
        L.mrf_net_forward_bf16.argtypes = [vp, vp, i64, vp, vp]
        L.mrf_net_loss_grad.argtypes = [vp, vp, vp, i64, ctypes.POINTER(ctypes.c_double), vp]
        L.mrf_net_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.mrf_net_noisy_batch.argtypes = [vp, vp, ctypes.c_uint64, i64, i64, ctypes.c_float,
                                          ctypes.c_float, vp, vp, vp, vp]
        L.mrf_net_train.argtypes = [vp, vp, ctypes.POINTER(TrainOpts), ctypes.POINTER(TrainStats), vp]
        L.mrf_op_forward.argtypes = [ctypes.POINTER(Op), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
        L.mrf_op_adjoint.argtypes = [ctypes.POINTER(Op), ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.mrf_ipg_step.argtypes = [ctypes.c_void_p, ctypes.POINTER(Op), ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                   ctypes.POINTER(MatchOpts), ctypes.POINTER(StepStats), ctypes.c_void_p]
        L.mrf_ipg_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Op), ctypes.c_void_p,
                                    ctypes.POINTER(SolveOpts), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SolveStats),
                                    ctypes.c_void_p]
        L.mrf_quantize_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        _LIB = L
    return _LIB


def _check(status):
    if status != MRF_OK:
        raise MrfError(status, lib().mrf_last_error().decode())


def _torch():
    import torch
    return torch


def _dev(t, dtype=None):
    """Device pointer of a CUDA tensor (None -> NULL), checking its dtype."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def mrf_version() -> str:
    return lib().mrf_version().decode()


# --------------------------------------------------------------------------- dictionary
class Dictionary:
    """Handle of a device dictionary (mrf_dict_build / mrf_dict_destroy)."""

    def __init__(self, atoms, params, grid_dims=None, store_bf16=False, store_fp8=False,
                 cover_tree=False, stream=None):
        atoms = np.asarray(atoms)
        self.is_complex = bool(np.iscomplexobj(atoms))
        d, L = atoms.shape
        if self.is_complex:
            if atoms.dtype == np.complex64:
                host = np.ascontiguousarray(atoms).view(np.float32)
                dt = MRF_F32
            else:
                host = np.ascontiguousarray(atoms.astype(np.complex128)).view(np.float64)
                dt = MRF_F64
        else:
            if atoms.dtype == np.float32:
                host, dt = np.ascontiguousarray(atoms), MRF_F32
            else:
                host, dt = np.ascontiguousarray(atoms, dtype=np.float64), MRF_F64
        params = np.ascontiguousarray(params, dtype=np.float64)
        if params.ndim == 1:
            params = params[:, None]
        self.nparam = params.shape[1]
        gd = None if grid_dims is None else np.ascontiguousarray(grid_dims, dtype=np.int32)
        flags = ((MRF_STORE_BF16 if store_bf16 else 0) | (MRF_STORE_FP8 if store_fp8 else 0)
                 | (MRF_BUILD_COVERTREE if cover_tree else 0))
        desc = DictDesc(d, L, self.nparam, int(self.is_complex), host.ctypes.data, dt,
                        params.ctypes.data, None if gd is None else gd.ctypes.data, flags)
        h = ctypes.c_void_p()
        _check(lib().mrf_dict_build(ctypes.byref(desc), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.d, self.L = d, L
        self.L_full = 0
        self.aligned = False
        self.grid_dims = None if gd is None else tuple(int(x) for x in gd)

    def compress(self, s, store_bf16=False, store_fp8=False, cover_tree=False, stream=None) -> "Dictionary":
        """mrf_dict_compress: a new dictionary of the s-frame compressed atoms
        V^H Dhat_j (V = the s dominant eigenvectors of sum_j Dhat_j Dhat_j^H)."""
        flags = ((MRF_STORE_BF16 if store_bf16 else 0) | (MRF_STORE_FP8 if store_fp8 else 0)
                 | (MRF_BUILD_COVERTREE if cover_tree else 0))
        h = ctypes.c_void_p()
        _check(lib().mrf_dict_compress(self.handle, int(s), flags, _stream(stream), ctypes.byref(h)))
        C = Dictionary.__new__(Dictionary)
        C.handle = h
        C.is_complex, C.nparam, C.d, C.L, C.L_full = True, self.nparam, self.d, int(s), self.L
        C.aligned = False
        C.grid_dims = self.grid_dims
        return C

    def align(self, store_bf16=False, store_fp8=False, cover_tree=False, stream=None) -> "Dictionary":
        """mrf_dict_align: a new dictionary of phase-aligned atoms for the
        complex-PD projection (keeps the temporal subspace of a compressed one)."""
        flags = ((MRF_STORE_BF16 if store_bf16 else 0) | (MRF_STORE_FP8 if store_fp8 else 0)
                 | (MRF_BUILD_COVERTREE if cover_tree else 0))
        h = ctypes.c_void_p()
        _check(lib().mrf_dict_align(self.handle, flags, _stream(stream), ctypes.byref(h)))
        C = Dictionary.__new__(Dictionary)
        C.handle = h
        C.is_complex, C.nparam, C.d, C.L, C.L_full = self.is_complex, self.nparam, self.d, self.L, self.L_full
        C.aligned = True
        C.grid_dims = self.grid_dims
        return C

    def subspace(self):
        """(V [L_full][s] complex128, eigenvalues [s]) of a compressed dictionary."""
        V = np.empty((self.L_full, self.L), dtype=np.complex128)
        lam = np.empty(self.L, dtype=np.float64)
        _check(lib().mrf_dict_subspace(self.handle, V.ctypes.data, lam.ctypes.data))
        return V, lam

    def info(self) -> DictInfo:
        inf = DictInfo()
        _check(lib().mrf_dict_query(self.handle, ctypes.byref(inf)))
        return inf

    def tree_info(self) -> TreeInfo:
        inf = TreeInfo()
        _check(lib().mrf_dict_tree_info(self.handle, ctypes.byref(inf)))
        return inf

    def tree_export(self):
        inf = self.tree_info()
        u = inf.unique_atoms
        rep = np.empty(u, np.int32)
        lev = np.empty(u, np.int32)
        par = np.empty(u, np.int32)
        md = np.empty(inf.entries, np.float32)
        _check(lib().mrf_dict_tree_export(self.handle, rep.ctypes.data, lev.ctypes.data, par.ctypes.data,
                                          md.ctypes.data))
        return dict(rep=rep, ins_level=lev, parent=par, maxdist=md, sigma=inf.sigma, imax=inf.imax)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().mrf_dict_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mrf_dict_copy_atoms(D: Dictionary, precision="fp32", stream=None):
    torch = _torch()
    inf = D.info()
    p = PRECISION[precision]
    dtype = {MRF_FP32: torch.float32, MRF_BF16: torch.int16, MRF_FP8: torch.uint8, MRF_BF16X3: torch.int16}[p]
    out = torch.empty((inf.d, 2 * inf.K if p == MRF_BF16X3 else inf.K), dtype=dtype, device="cuda")
    scales = torch.empty(inf.d, dtype=torch.float32, device="cuda") if p == MRF_FP8 else None
    _check(lib().mrf_dict_copy_atoms(D.handle, p, _dev(out), _dev(scales), _stream(stream)))
    return (out, scales) if p == MRF_FP8 else out


def match_opts(precision="fp32", topk=8, atom_splits=0, net=None, box_radius=3, fallback_corr=0.98,
               recentre=0, eps=None, tree_capacity=0, certify=True, certify_local=False) -> MatchOpts:
    # a network selects the learned path (a given eps then sends its fallback
    # voxels to the dictionary's cover tree, None keeps the exhaustive
    # fallback); eps alone selects the cover tree
    if net is not None:
        method = MRF_LEARNED
        e = -1.0 if eps is None else float(eps)
    else:
        method = MRF_COVERTREE if eps is not None else MRF_EXHAUSTIVE
        e = float(eps or 0.0)
    return MatchOpts(method, PRECISION[precision], int(topk), int(atom_splits),
                     None if net is None else net.handle, int(box_radius), float(fallback_corr),
                     int(recentre), e, int(tree_capacity), None, 0 if certify else 1, 1 if certify_local else 0)


# --------------------------------------------------------------------------- matched filter
def mrf_match(D: Dictionary, Z, layout="voxel", slice_voxels=None, precision="fp32", topk=8,
              atom_splits=0, warm_idx=None, want_pd=True, want_corr=True, want_X=False,
              want_params=False, stats=False, out=None, stream=None, net=None, box_radius=3,
              fallback_corr=0.98, recentre=0, eps=None, tree_capacity=0, want_pd_phase=False, certify=True,
              certify_local=False):
    """Matched filter of the voxels in Z (complex64 CUDA tensor, [n][L] for
    layout 'voxel', [S][L][...] for 'frame').  Returns a dict of CUDA tensors
    (idx, pd, corr, X, params, pd_phase) and, with stats=True, a MatchStats.
    certify=False skips the exhaustive filter's exactness certificate;
    certify_local=True makes the learned path's local search exact (FP64
    argmax over each voxel's box and warm atom)."""
    torch = _torch()
    if layout == "voxel":
        n = Z.shape[0]
        zl, sv = MRF_VOXEL_MAJOR, 0
    else:
        sv = int(slice_voxels) if slice_voxels is not None else int(np.prod(Z.shape[2:]))
        n = int(Z.numel() // D.L)
        zl = MRF_FRAME_MAJOR
    o = out if out is not None else {}
    dev = Z.device
    if "idx" not in o:
        o["idx"] = torch.empty(n, dtype=torch.int32, device=dev)
    if want_pd and "pd" not in o:
        o["pd"] = torch.empty(n, dtype=torch.float32, device=dev)
    if want_corr and "corr" not in o:
        o["corr"] = torch.empty(n, dtype=torch.float32, device=dev)
    if want_X and "X" not in o:
        o["X"] = torch.empty_like(Z)
    if want_params and "params" not in o:
        o["params"] = torch.empty((n, D.nparam), dtype=torch.float32, device=dev)
    opts = match_opts(precision, topk, atom_splits, net, box_radius, fallback_corr, recentre, eps,
                      tree_capacity, certify, certify_local)
    if want_pd_phase:
        if "pd_phase" not in o:
            o["pd_phase"] = torch.empty(n, dtype=torch.float32, device=dev)
        opts.pd_phase = _dev(o["pd_phase"])
    st = MatchStats() if stats else None
    status = lib().mrf_match(D.handle, ctypes.byref(opts), n, _dev(Z, torch.complex64), zl, sv,
                             _dev(warm_idx, torch.int32),
                             _dev(o["idx"]), _dev(o.get("pd")), _dev(o.get("corr")),
                             _dev(o.get("X")), _dev(o.get("params")),
                             ctypes.byref(st) if st is not None else None, _stream(stream))
    _check(status)
    if stats:
        o["stats"] = st
    return o


def mrf_match_noalloc(D: Dictionary, Z, out, layout="voxel", slice_voxels=None, atom_splits=0, warm_idx=None,
                      certify=True, stream=None):
    """mrf_match_noalloc: the exhaustive FP32 filter on the library's fixed
    workspace (no device allocation).  `out` holds the caller's CUDA tensors
    idx (required), pd, corr, X, params (optional)."""
    torch = _torch()
    if layout == "voxel":
        n, zl, sv = Z.shape[0], MRF_VOXEL_MAJOR, 0
    else:
        sv = int(slice_voxels) if slice_voxels is not None else int(np.prod(Z.shape[2:]))
        n, zl = int(Z.numel() // D.L), MRF_FRAME_MAJOR
    opts = match_opts("fp32", 8, atom_splits, certify=certify)
    _check(lib().mrf_match_noalloc(D.handle, ctypes.byref(opts), n, _dev(Z, torch.complex64), zl, sv,
                                   _dev(warm_idx, torch.int32), _dev(out["idx"]), _dev(out.get("pd")),
                                   _dev(out.get("corr")), _dev(out.get("X")), _dev(out.get("params")),
                                   _stream(stream)))
    return out


def mrf_match_local(D: Dictionary, Z, cells, layout="voxel", slice_voxels=None, box_radius=3,
                    fallback_corr=0.98, recentre=0, warm_idx=None, want_X=False, want_params=False,
                    stats=False, stream=None, precision="fp32", certify_local=False):
    """Local matched filter around given proposal cells (int32 CUDA tensor
    [n][nparam], modified in place by re-centring); certify_local=True makes
    it exact (FP64 argmax over each box and warm atom)."""
    torch = _torch()
    if layout == "voxel":
        n, zl, sv = Z.shape[0], MRF_VOXEL_MAJOR, 0
    else:
        sv = int(slice_voxels) if slice_voxels is not None else int(np.prod(Z.shape[2:]))
        n, zl = int(Z.numel() // D.L), MRF_FRAME_MAJOR
    dev = Z.device
    o = {"idx": torch.empty(n, dtype=torch.int32, device=dev),
         "pd": torch.empty(n, dtype=torch.float32, device=dev),
         "corr": torch.empty(n, dtype=torch.float32, device=dev),
         "fallback": torch.empty(n, dtype=torch.int32, device=dev)}
    if want_X:
        o["X"] = torch.empty_like(Z)
    if want_params:
        o["params"] = torch.empty((n, D.nparam), dtype=torch.float32, device=dev)
    opts = match_opts(precision, 8, 0, None, box_radius, fallback_corr, recentre, None, 0,
                      certify_local=certify_local)
    st = MatchStats() if stats else None
    _check(lib().mrf_match_local(D.handle, ctypes.byref(opts), n, _dev(Z, torch.complex64), zl, sv,
                                 _dev(cells, torch.int32), _dev(warm_idx, torch.int32), _dev(o["idx"]), _dev(o["pd"]), _dev(o["corr"]),
                                 _dev(o["fallback"]), _dev(o.get("X")), _dev(o.get("params")),
                                 ctypes.byref(st) if st is not None else None, _stream(stream)))
    if stats:
        o["stats"] = st
    return o


# --------------------------------------------------------------------------- network
class Net:
    """Handle of a learned proposal network (mrf_net_create / mrf_net_destroy)."""

    def __init__(self, in_dim, nout, hidden=256, seed=0):
        h = ctypes.c_void_p()
        _check(lib().mrf_net_create(int(in_dim), int(hidden), int(nout), int(seed), ctypes.byref(h)))
        self.handle = h
        self.in_dim, self.hidden, self.nout = int(in_dim), int(hidden), int(nout)
        c = ctypes.c_int64()
        _check(lib().mrf_net_size(h, ctypes.byref(c)))
        self.size = c.value

    def offsets(self):
        I, H, P = self.in_dim, self.hidden, self.nout
        o = {"W1": (0, (H, I))}
        o["b1"] = (H * I, (H,))
        o["W2"] = (H * I + H, (H, H))
        o["b2"] = (H * I + H + H * H, (H,))
        o["W3"] = (H * I + 2 * H + H * H, (P, H))
        o["b3"] = (H * I + 2 * H + H * H + P * H, (P,))
        return o

    def get_params(self):
        a = np.empty(self.size, dtype=np.float32)
        _check(lib().mrf_net_get_params(self.handle, a.ctypes.data, self.size))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        _check(lib().mrf_net_set_params(self.handle, a.ctypes.data, a.size))

    def get_grads(self):
        a = np.empty(self.size, dtype=np.float32)
        _check(lib().mrf_net_get_grads(self.handle, a.ctypes.data, self.size))
        return a

    def unpack(self, flat):
        return {k: np.asarray(flat[o:o + int(np.prod(sh))]).reshape(sh) for k, (o, sh) in self.offsets().items()}

    def set_standardisation(self, mean, std, log_mask):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        lm = np.ascontiguousarray(log_mask, dtype=np.int32)
        _check(lib().mrf_net_set_standardisation(self.handle, m.ctypes.data, s.ctypes.data, lm.ctypes.data))

    def get_standardisation(self):
        m = np.empty(self.nout, np.float32)
        s = np.empty(self.nout, np.float32)
        lm = np.empty(self.nout, np.int32)
        _check(lib().mrf_net_get_standardisation(self.handle, m.ctypes.data, s.ctypes.data, lm.ctypes.data))
        return m, s, lm

    def save(self, path):
        """Weights and output standardisation to a .npz file (no pickles)."""
        m, sd, lm = self.get_standardisation()
        np.savez(path, dims=np.array([self.in_dim, self.hidden, self.nout], dtype=np.int64),
                 params=self.get_params(), mean=m, std=sd, log_mask=lm)

    @classmethod
    def load(cls, path):
        """A network saved by save()."""
        with np.load(path, allow_pickle=False) as f:
            I, H, P = (int(x) for x in f["dims"])
            net = cls(I, P, hidden=H)
            net.set_params(f["params"])
            net.set_standardisation(f["mean"], f["std"], f["log_mask"])
        return net

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().mrf_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mrf_net_forward(net: Net, X, stream=None, bf16=False):
    """Y = net(X) in FP32, or (bf16=True) in the BF16 inference form the
    learned match uses for its proposal."""
    torch = _torch()
    Y = torch.empty((X.shape[0], net.nout), dtype=torch.float32, device="cuda")
    fn = lib().mrf_net_forward_bf16 if bf16 else lib().mrf_net_forward
    _check(fn(net.handle, _dev(X, torch.float32), X.shape[0], _dev(Y), _stream(stream)))
    return Y


def mrf_net_loss_grad(net: Net, X, T, stream=None):
    loss = ctypes.c_double()
    torch = _torch()
    _check(lib().mrf_net_loss_grad(net.handle, _dev(X, torch.float32), _dev(T, torch.float32), X.shape[0], ctypes.byref(loss),
                                   _stream(stream)))
    return loss.value


def mrf_net_adam(net: Net, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().mrf_net_adam(net.handle, lr, beta1, beta2, eps, _stream(stream)))


def mrf_net_noisy_batch(net: Net, D: Dictionary, seed, offset, B, snr_lo=15.0, snr_hi=40.0,
                        stream=None):
    torch = _torch()
    K = D.info().K
    X = torch.empty((B, K), dtype=torch.float32, device="cuda")
    T = torch.empty((B, net.nout), dtype=torch.float32, device="cuda")
    A = torch.empty(B, dtype=torch.int32, device="cuda")
    _check(lib().mrf_net_noisy_batch(net.handle, D.handle, int(seed), int(offset), int(B), snr_lo,
                                     snr_hi, _dev(X), _dev(T), _dev(A), _stream(stream)))
    return X, T, A


def mrf_net_train(net: Net, D: Dictionary, samples=2_000_000, batch=4096, epochs=4, lr=1e-3,
                  lr_min=1e-5, snr_lo=15.0, snr_hi=40.0, seed=1, stream=None):
    o = TrainOpts(int(samples), int(batch), int(epochs), float(lr), float(lr_min), float(snr_lo),
                  float(snr_hi), int(seed))
    st = TrainStats()
    _check(lib().mrf_net_train(net.handle, D.handle, ctypes.byref(o), ctypes.byref(st), _stream(stream)))
    return dict(steps=st.steps, first_loss=st.first_loss, last_loss=st.last_loss, ms=st.ms)


# --------------------------------------------------------------------------- operator
class Nufft:
    """Non-uniform FFT plan of a non-Cartesian trajectory (mrf_nufft_create)."""

    def __init__(self, nx, ny, L, nslices, samp_off, coords, width=0):
        off = np.ascontiguousarray(samp_off, dtype=np.int64)
        k = np.ascontiguousarray(coords, dtype=np.float32)
        h = ctypes.c_void_p()
        _check(lib().mrf_nufft_create(int(nx), int(ny), int(L), int(nslices), int(off[-1]), off.ctypes.data,
                                      k.ctypes.data, int(width), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().mrf_nufft_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """mrf_op over device copies of a CSR sampling pattern (see include/mrf.h)."""

    def __init__(self, nx, ny, L, nslices, samp_off, samp_idx, dcf=None, smaps=None, nufft=None):
        """smaps: coil sensitivity maps [nslices][c][ny][nx] (complex), or None
        for one coil with S = I; with c coils the sample arrays are [c][M].
        nufft: a Nufft plan for non-Cartesian samples (samp_idx unused)."""
        torch = _torch()
        self.off = torch.as_tensor(np.asarray(samp_off, dtype=np.int64)).cuda()
        self.nufft = nufft
        if samp_idx is None:
            samp_idx = np.zeros(0, dtype=np.int32)
        self.idx = torch.as_tensor(np.asarray(samp_idx, dtype=np.int32)).cuda()
        self.dcf = None if dcf is None else torch.as_tensor(np.asarray(dcf, dtype=np.float32)).cuda()
        self.nx, self.ny, self.L, self.nslices = int(nx), int(ny), int(L), int(nslices)
        self.M = int(self.off[-1].item()) if self.off.numel() else 0
        self.smaps = None
        self.ncoils = 0
        if smaps is not None:
            sm = np.ascontiguousarray(np.asarray(smaps).astype(np.complex64))
            assert sm.ndim == 4 and sm.shape[0] == self.nslices and sm.shape[2:] == (self.ny, self.nx)
            self.smaps = torch.from_numpy(sm).cuda()
            self.ncoils = int(sm.shape[1])
        self.c = Op(self.nx, self.ny, self.L, self.nslices, self.M, _dev(self.off),
                    _dev(self.idx) if self.idx.numel() else None, _dev(self.dcf), self.ncoils, 0,
                    _dev(self.smaps), None if nufft is None else nufft.handle)

    @property
    def n(self):
        return self.nslices * self.nx * self.ny

    @property
    def nsamp(self):
        """Samples per sample array: M, or c*M with c coils (coil-major)."""
        return max(self.ncoils, 1) * self.M

    @classmethod
    def from_sampling(cls, smp, smaps=None):
        return cls(smp.nx, smp.ny, smp.L, smp.S, smp.off, smp.idx, smp.dcf, smaps=smaps)

    @classmethod
    def from_trajectory(cls, tr, smaps=None, width=0, dcf=True):
        """Non-Cartesian operator of a trajectory (coords [M][2] (ky, kx) in
        cycles per pixel, CSR offsets per (slice, frame))."""
        plan = Nufft(tr.nx, tr.ny, tr.L, tr.S, tr.off, tr.coords, width)
        return cls(tr.nx, tr.ny, tr.L, tr.S, tr.off, None, tr.dcf if dcf else None, smaps=smaps, nufft=plan)


def mrf_op_forward(A: Operator, X, Y=None, want_norm=False, stream=None):
    torch = _torch()
    R = torch.empty(max(A.nsamp, 1), dtype=torch.complex64, device="cuda")[:A.nsamp]
    if A.ncoils:
        R = R.view(A.ncoils, A.M)
    nrm = ctypes.c_double(0.0)
    _check(lib().mrf_op_forward(ctypes.byref(A.c), _dev(X), _dev(Y), R.data_ptr(),
                                ctypes.byref(nrm) if want_norm else None, _stream(stream)))
    return (R, nrm.value) if want_norm else R


def mrf_op_adjoint(A: Operator, R, apply_dcf=True, stream=None):
    torch = _torch()
    G = torch.empty((A.nslices, A.L, A.ny, A.nx), dtype=torch.complex64, device="cuda")
    _check(lib().mrf_op_adjoint(ctypes.byref(A.c), R.data_ptr() if A.M else None,
                                int(bool(apply_dcf)), _dev(G), _stream(stream)))
    return G


# --------------------------------------------------------------------------- projected gradient
def mrf_ipg_step(D: Dictionary, A: Operator, Y, X_in, mu, idx_in=None, precision="fp32", topk=8,
                 atom_splits=0, stats=True, stream=None, net=None, box_radius=3, fallback_corr=0.98,
                 recentre=0, eps=None, tree_capacity=0, certify=True, certify_local=False):
    torch = _torch()
    X_out = torch.empty_like(X_in)
    idx = torch.empty(A.n, dtype=torch.int32, device="cuda")
    pd = torch.empty(A.n, dtype=torch.float32, device="cuda")
    opts = match_opts(precision, topk, atom_splits, net, box_radius, fallback_corr, recentre, eps, tree_capacity,
                      certify, certify_local)
    st = StepStats() if stats else None
    _check(lib().mrf_ipg_step(D.handle, ctypes.byref(A.c), _dev(Y), _dev(X_in), _dev(X_out),
                              _dev(idx_in), _dev(idx), _dev(pd), float(mu), ctypes.byref(opts),
                              ctypes.byref(st) if st is not None else None, _stream(stream)))
    return X_out, idx, pd, st


def mrf_ipg_solve(D: Dictionary, A: Operator, Y, X0=None, mu0=1.0, zeta=2.0, adaptive=True,
                  max_iter=50, rel_tol=1e-6, max_shrinks=30, kappa=False, precision="fp32",
                  topk=8, atom_splits=0, want_params=True, stream=None, net=None, box_radius=3,
                  fallback_corr=0.98, recentre=0, eps=None, tree_capacity=0, certify=True, certify_local=False):
    """Algorithm 2.  The projection is exhaustive (default), learned (net
    given: proposal + local search + fallback, warm-started by the previous
    iterate's atoms) or the cover tree (eps given)."""
    torch = _torch()
    X = (torch.zeros((A.nslices, D.L, A.ny, A.nx), dtype=torch.complex64, device="cuda")
         if X0 is None else X0.clone())
    idx = torch.empty(A.n, dtype=torch.int32, device="cuda")
    pd = torch.empty(A.n, dtype=torch.float32, device="cuda")
    params = torch.empty((A.n, D.nparam), dtype=torch.float32, device="cuda") if want_params else None
    o = SolveOpts(float(mu0), float(zeta), int(bool(adaptive)), int(max_iter), float(rel_tol),
                  int(max_shrinks), int(bool(kappa)),
                  match_opts(precision, topk, atom_splits, net, box_radius, fallback_corr, recentre, eps,
                             tree_capacity, certify, certify_local))
    cap = int(max_iter)
    f = np.zeros(cap, dtype=np.float64)
    mu = np.zeros(cap, dtype=np.float32)
    sh = np.zeros(cap, dtype=np.int32)
    st = SolveStats(0, 0, cap, f.ctypes.data, mu.ctypes.data, sh.ctypes.data, 0.0, 0.0, 0)
    _check(lib().mrf_ipg_solve(D.handle, ctypes.byref(A.c), _dev(Y), ctypes.byref(o), _dev(X),
                               _dev(idx), _dev(pd), _dev(params), ctypes.byref(st), _stream(stream)))
    k = st.iters
    hist = dict(iters=k, total_shrinks=st.total_shrinks, f0=st.f0, f=f[:k].copy(), mu=mu[:k].copy(),
                shrinks=sh[:k].copy(), ms=st.ms, fallbacks=st.fallbacks,
                distance_evals=st.distance_evals)
    return X, idx, pd, params, hist


# --------------------------------------------------------------------------- encodings
def mrf_quantize_rows(x, precision, out_pitch=None, stream=None):
    """Encode FP32 rows (2-D CUDA tensor) to BF16 (int16 bit patterns) or FP8
    (uint8 codes + per-row scales)."""
    torch = _torch()
    rows, K = x.shape
    pitch = int(out_pitch or K)
    p = PRECISION[precision]
    if p == MRF_BF16:
        out = torch.empty((rows, pitch), dtype=torch.int16, device="cuda")
        sc = None
    else:
        out = torch.empty((rows, pitch), dtype=torch.uint8, device="cuda")
        sc = torch.empty(rows, dtype=torch.float32, device="cuda")
    _check(lib().mrf_quantize_rows(_dev(x), rows, K, x.stride(0), p, _dev(out), pitch, _dev(sc),
                                   _stream(stream)))
    return out, sc

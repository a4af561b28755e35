"""ctypes binding of libris_hip.so (the C ABI in include/ris.h).

Argument marshalling only: every step of the path runs in the library's gfx950
kernels.  Large arrays are torch CUDA (HIP) tensors whose device pointers are
handed to the library; the context enqueues on torch's current stream of the
tensors' device.  There is no fallback: without the built library or without a
GPU every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libris_hip.so")

RIS_OK = 0
STATUS = {0: "RIS_OK", 1: "RIS_E_INVALID", 2: "RIS_E_UNSUPPORTED", 3: "RIS_E_NOMEM", 4: "RIS_E_NOT_PD",
          5: "RIS_E_DEGENERATE", 6: "RIS_E_ORDER", 7: "RIS_E_DEVICE", 8: "RIS_E_NOCONV"}
OPS = {"A": 0, "B": 1, "A+B": 2, "A-B": 3}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
PREC_TRANSFORMS = 16  # or-ed into a mode: the MO transforms of (mu nu|P) run in it too
DENSITY = {"ground": 0, "difference": 1, "relaxed": 2}
EXPORTS = ("ris_ctx_create", "ris_ctx_destroy", "ris_last_error", "ris_ctx_bytes", "ris_ctx_release", "ris_aux_build", "ris_int3c",
           "ris_response_matvec", "ris_response_matvec_noalloc", "ris_grad_contract", "ris_nac_contract", "ris_grad_nac_contract",
           "ris_request_bytes", "ris_plan_bytes",
           "ris_ctx_set_profiling", "ris_ctx_set_screening", "ris_ctx_set_blocking", "ris_zvector_solve",
           "ris_tda_davidson",
           "ris_zrhs_contract", "ris_density_ao",
           "ris_ctx_stage_stats",
           # test-only building blocks (include/ris_test.h)
           "ris_test_mfma_probe", "ris_test_dgemm", "ris_test_gemm", "ris_test_sym_eig",
           "ris_test_transpose", "ris_test_boys", "ris_test_pgemm")


class RisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class _Mol(ctypes.Structure):
    _fields_ = [("natm", ctypes.c_int), ("Z", ctypes.POINTER(ctypes.c_int)),
                ("xyz", ctypes.POINTER(ctypes.c_double)), ("nshell", ctypes.c_int),
                ("shell_atom", ctypes.POINTER(ctypes.c_int)), ("shell_l", ctypes.POINTER(ctypes.c_int)),
                ("shell_exp", ctypes.POINTER(ctypes.c_double))]


class _AuxOpts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("radius_bohr", ctypes.POINTER(ctypes.c_double)),
                ("j_p_on_heavy", ctypes.c_int)]


class _MO(ctypes.Structure):
    _fields_ = [("nao", ctypes.c_int), ("nmo", ctypes.c_int), ("nocc", ctypes.c_int),
                ("C", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("alpha_J", ctypes.c_double),
                ("c_x", ctypes.c_double), ("precision", ctypes.c_int)]


class _Extra(ctypes.Structure):
    _fields_ = [("out", ctypes.c_int), ("D1", ctypes.c_void_p), ("D2", ctypes.c_void_p), ("cJ", ctypes.c_double),
                ("cK", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libris_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2511_18233_amd.build`")
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    lib.ris_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_size_t]
    lib.ris_ctx_destroy.argtypes = [vp]
    lib.ris_ctx_destroy.restype = None
    lib.ris_last_error.argtypes = [vp]
    lib.ris_last_error.restype = ctypes.c_char_p
    lib.ris_ctx_bytes.argtypes = [vp]
    lib.ris_ctx_bytes.restype = ctypes.c_size_t
    lib.ris_ctx_release.argtypes = [vp]
    lib.ris_aux_build.argtypes = [vp, ctypes.POINTER(_Mol), ctypes.POINTER(_AuxOpts), ip, ip]
    lib.ris_int3c.argtypes = [vp, ctypes.POINTER(_MO), vp]
    lib.ris_response_matvec.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.ris_response_matvec_noalloc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp]
    ep = ctypes.POINTER(_Extra)
    lib.ris_grad_contract.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ip, ctypes.c_int, ep, vp]
    lib.ris_nac_contract.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ip, ctypes.c_int, ep, dp, vp]
    lib.ris_density_ao.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.ris_request_bytes.argtypes = [ctypes.POINTER(_Mol), ctypes.POINTER(_AuxOpts), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.ris_request_bytes.restype = ctypes.c_size_t
    lib.ris_plan_bytes.argtypes = [ctypes.POINTER(_Mol), ctypes.POINTER(_AuxOpts), ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.ris_plan_bytes.restype = ctypes.c_size_t
    lib.ris_grad_nac_contract.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ip, vp, ctypes.c_int, ip, dp, vp,
                                          ctypes.c_int, ep]
    lib.ris_ctx_set_profiling.argtypes = [vp, ctypes.c_int]
    lib.ris_ctx_set_screening.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_long)]
    lib.ris_ctx_set_blocking.argtypes = [vp, ctypes.c_int]
    lib.ris_zvector_solve.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_double, ctypes.c_int, ip, dp]
    lib.ris_tda_davidson.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, vp, ip]
    lib.ris_zrhs_contract.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int, ip, vp]
    lib.ris_ctx_stage_stats.argtypes = [vp, ctypes.c_int, dp, dp, dp, ctypes.POINTER(ctypes.c_long)]
    lib.ris_test_mfma_probe.argtypes = [ctypes.c_int, vp, vp, vp]
    L = ctypes.c_long
    lib.ris_test_dgemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_double, vp, L, L, vp, L, L, ctypes.c_double, vp, L, L, ctypes.c_int]
    lib.ris_test_gemm.argtypes = [ctypes.c_int] + lib.ris_test_dgemm.argtypes
    lib.ris_test_sym_eig.argtypes = [ctypes.c_int, vp, vp]
    lib.ris_test_transpose.argtypes = [vp, L, vp, L, ctypes.c_int, ctypes.c_int]
    lib.ris_test_boys.argtypes = [ctypes.c_int, vp, vp]
    lib.ris_test_pgemm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, vp,
                                   ctypes.c_long, vp, ctypes.c_long, ctypes.c_double, vp, ctypes.c_long,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    _lib = lib
    return lib


def request_bytes(Z, shell_atom, shell_l, radius_bohr, nmo, nocc, nstate, nvec=0, nout=0, theta=0.2,
                  j_p_on_heavy=True, aux_block=0, xyz=None, shell_exp=None) -> int:
    """Device bytes one request needs (host-only sizing from the library);
    aux_block > 0: the footprint of the path blocked over the auxiliary index.
    xyz (Bohr) and shell_exp size the screened AO shell pairs; without them
    every pair counts as kept (an upper bound)."""
    lib = load_library()
    Z = np.ascontiguousarray(Z, dtype=np.int32)
    sa = np.ascontiguousarray(shell_atom, dtype=np.int32)
    sl = np.ascontiguousarray(shell_l, dtype=np.int32)
    se = np.ones(sl.shape[0]) if shell_exp is None else np.ascontiguousarray(shell_exp, dtype=np.float64)
    xyz = np.zeros((Z.shape[0], 3)) if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
    rad = np.ascontiguousarray(radius_bohr, dtype=np.float64)
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    mol = _Mol(Z.shape[0], Z.ctypes.data_as(ip), xyz.ctypes.data_as(dp), sl.shape[0], sa.ctypes.data_as(ip),
               sl.ctypes.data_as(ip), se.ctypes.data_as(dp))
    opts = _AuxOpts(float(theta), rad.ctypes.data_as(dp), int(bool(j_p_on_heavy)))
    return int(lib.ris_plan_bytes(ctypes.byref(mol), ctypes.byref(opts), int(nmo), int(nocc), int(nstate),
                                  int(nvec), int(nout), int(aux_block)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _extra_array(extra, dev, nao):
    """(count, ctypes array) of ris_extra_pair from [(out, D1, D2, cJ, cK)]
    with D1, D2 device float64 [nao][nao] tensors."""
    if not extra:
        return 0, None
    arr = (_Extra * len(extra))()
    for k, (out, D1, D2, cJ, cK) in enumerate(extra):
        for nm, D in (("D1", D1), ("D2", D2)):
            _check_dev(D, dev, f"extra[{k}].{nm}")
            if tuple(D.shape) != (nao, nao):
                raise ValueError(f"extra[{k}].{nm} must be [{nao}][{nao}]")
        arr[k] = _Extra(int(out), D1.data_ptr(), D2.data_ptr(), float(cJ), float(cK))
    return len(extra), arr


def _check_dev(t, dev, name):
    import torch
    if t is None:
        return
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
    if t.device != dev:
        raise ValueError(f"{name} is on {t.device}, context on {dev}")


class RisContext:
    """One library context on one GPU (torch device), enqueueing on a stream."""

    def __init__(self, device=0, stream=None, hbm_budget: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ris library runs on MI355X only")
        self.lib = load_library()
        self.device = torch.device("cuda", device if isinstance(device, int) else torch.device(device).index or 0)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.ris_ctx_create(ctypes.byref(h), self.device.index, ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.c_size_t(hbm_budget))
        if st != RIS_OK:
            raise RisError(st, "ris_ctx_create failed")
        self.h = h
        self.natm = self.nao = 0
        self.nJ = self.nK = 0
        self.nocc = self.nvir = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.ris_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != RIS_OK:
            raise RisError(st, self.lib.ris_last_error(self.h).decode())

    @property
    def bytes_held(self) -> int:
        return int(self.lib.ris_ctx_bytes(self.h))

    def release(self):
        """Free the context's request regions (ris_ctx_release)."""
        self._chk(self.lib.ris_ctx_release(self.h))

    STAGES = ("int3c", "mo", "matvec", "hblk", "gamma", "deriv", "aux", "yw", "vpq")

    def set_screening(self, threshold: float) -> int:
        """Shell-pair screen threshold of the derivative contraction (0: off);
        returns the number of ordered shell pairs kept (-1 before aux_build)."""
        kept = ctypes.c_long(0)
        self._chk(self.lib.ris_ctx_set_screening(self.h, float(threshold), ctypes.byref(kept)))
        return int(kept.value)

    def set_blocking(self, aux_block: int):
        """Cap on auxiliary functions per block (0: unblocked when it fits,
        else the largest blocks that fit the HBM budget)."""
        self._chk(self.lib.ris_ctx_set_blocking(self.h, int(aux_block)))

    def set_profiling(self, on: bool):
        self._chk(self.lib.ris_ctx_set_profiling(self.h, int(bool(on))))

    def stage_stats(self):
        """{stage: (ms, flops, bytes, launches)} accumulated since profiling was enabled."""
        out = {}
        for k, name in enumerate(self.STAGES):
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            n = ctypes.c_long()
            self._chk(self.lib.ris_ctx_stage_stats(self.h, k, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by),
                                                   ctypes.byref(n)))
            out[name] = (ms.value, fl.value, by.value, n.value)
        return out

    # -- entry points -----------------------------------------------------
    def aux_build(self, Z, xyz, shell_atom, shell_l, shell_exp, radius_bohr, theta=0.2, j_p_on_heavy=True):
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        sa = np.ascontiguousarray(shell_atom, dtype=np.int32)
        sl = np.ascontiguousarray(shell_l, dtype=np.int32)
        se = np.ascontiguousarray(shell_exp, dtype=np.float64)
        rad = np.ascontiguousarray(radius_bohr, dtype=np.float64)
        ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        mol = _Mol(Z.shape[0], Z.ctypes.data_as(ip), xyz.ctypes.data_as(dp), sl.shape[0], sa.ctypes.data_as(ip),
                   sl.ctypes.data_as(ip), se.ctypes.data_as(dp))
        opts = _AuxOpts(float(theta), rad.ctypes.data_as(dp), int(bool(j_p_on_heavy)))
        nJ, nK = ctypes.c_int(), ctypes.c_int()
        self._chk(self.lib.ris_aux_build(self.h, ctypes.byref(mol), ctypes.byref(opts), ctypes.byref(nJ),
                                         ctypes.byref(nK)))
        self.natm = int(Z.shape[0])
        self.nao = int(sum((l + 1) * (l + 2) // 2 for l in sl))
        self.nJ, self.nK = nJ.value, nK.value
        return self.nJ, self.nK

    def int3c(self, C, eps, nocc, alpha_J=2.0, c_x=0.25, precision=0, dbg=None):
        _check_dev(C, self.device, "C")
        _check_dev(eps, self.device, "eps")
        _check_dev(dbg, self.device, "dbg")
        nao, nmo = C.shape
        if isinstance(precision, str):
            # "fp32", or "fp32+transforms" for the MO transforms in the mode too
            base, _, tr = precision.partition("+")
            if base not in PRECISION or tr not in ("", "transforms"):
                raise ValueError(f"unknown precision {precision!r}")
            precision = PRECISION[base] | (PREC_TRANSFORMS if tr else 0)
        mo = _MO(nao, nmo, int(nocc), C.data_ptr(), eps.data_ptr(), float(alpha_J), float(c_x), int(precision))
        self._chk(self.lib.ris_int3c(self.h, ctypes.byref(mo), _ptr(dbg)))
        self.nocc, self.nvir = int(nocc), int(nmo - nocc)

    def response_matvec(self, op, V, out=None):
        import torch
        _check_dev(V, self.device, "V")
        if out is None:
            out = torch.empty_like(V)
        _check_dev(out, self.device, "out")
        nvec = V.shape[0] if V.dim() == 3 else 1
        self._chk(self.lib.ris_response_matvec(self.h, OPS[op] if isinstance(op, str) else int(op), nvec, _ptr(V),
                                               _ptr(out)))
        return out

    def response_matvec_noalloc(self, op, V, out):
        """ris_response_matvec_noalloc: the same product with the library's fixed
        device scratch (no allocation; enqueued only).  `out` must be given."""
        _check_dev(V, self.device, "V")
        _check_dev(out, self.device, "out")
        nvec = V.shape[0] if V.dim() == 3 else 1
        self._chk(self.lib.ris_response_matvec_noalloc(self.h, OPS[op] if isinstance(op, str) else int(op), nvec,
                                                       _ptr(V), _ptr(out)))
        return out

    def zvector_solve(self, rhs, tol=1e-10, maxit=200, out=None, allow_noconv=False):
        """(A+B)^ris Z = rhs for rhs[nrhs][nvir][nocc] (device FP64); returns
        (Z, iterations, largest true relative residual).  RIS_E_NOCONV raises
        unless allow_noconv."""
        import torch
        _check_dev(rhs, self.device, "rhs")
        if out is None:
            out = torch.empty_like(rhs)
        _check_dev(out, self.device, "Z")
        nrhs = rhs.shape[0] if rhs.dim() == 3 else 1
        it, res = ctypes.c_int(0), ctypes.c_double(0.0)
        st = self.lib.ris_zvector_solve(self.h, nrhs, _ptr(rhs), _ptr(out), float(tol), int(maxit), ctypes.byref(it),
                                        ctypes.byref(res))
        if not (st == 8 and allow_noconv):
            self._chk(st)
        return out, int(it.value), float(res.value)

    def zrhs_contract(self, X, Y, pairs, out=None):
        """ris terms of the Z-vector right-hand side per pair (I, J) as device
        [npair][nmo][nmo] MO matrices (gradient form for I == J)."""
        import torch
        _check_dev(X, self.device, "X")
        _check_dev(Y, self.device, "Y")
        pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        nmo = self.nocc + self.nvir
        if out is None:
            out = torch.empty((pr.shape[0], nmo, nmo), dtype=torch.float64, device=self.device)
        _check_dev(out, self.device, "G")
        self._chk(self.lib.ris_zrhs_contract(self.h, X.shape[0], _ptr(X), _ptr(Y), pr.shape[0],
                                             pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(out)))
        return out

    def tda_davidson(self, nroots, tol=1e-8, maxit=100, max_space=0, out=None, allow_noconv=False):
        """Lowest nroots TDA-ris eigenpairs: (omega numpy[nroots], X device
        [nroots][nvir][nocc], iterations).  RIS_E_NOCONV raises unless
        allow_noconv."""
        import torch
        if out is None:
            out = torch.empty((int(nroots), self.nvir, self.nocc), dtype=torch.float64, device=self.device)
        _check_dev(out, self.device, "X")
        w = np.zeros(int(nroots))
        it = ctypes.c_int(0)
        st = self.lib.ris_tda_davidson(self.h, int(nroots), float(tol), int(maxit), int(max_space),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(out), ctypes.byref(it))
        if not (st == 8 and allow_noconv):
            self._chk(st)
        return w, out, int(it.value)

    def density_ao(self, kind, X=None, Y=None, I=0, J=0, Z=None, out=None):
        """AO density [nao][nao] on the device: "ground" (C_O C_O^T), "difference"
        (T_IJ) or "relaxed" (T_IJ + Z^S, Z device [nvir][nocc])."""
        import torch
        _check_dev(X, self.device, "X")
        _check_dev(Y, self.device, "Y")
        _check_dev(Z, self.device, "Z")
        if out is None:
            out = torch.empty((self.nao, self.nao), dtype=torch.float64, device=self.device)
        _check_dev(out, self.device, "D")
        ns = X.shape[0] if X is not None else 0
        self._chk(self.lib.ris_density_ao(self.h, DENSITY[kind] if isinstance(kind, str) else int(kind), ns, _ptr(X),
                                          _ptr(Y), int(I), int(J), _ptr(Z), _ptr(out)))
        return out

    def grad_contract(self, X, Y, sel, out=None, extra=None):
        """Gradients of states sel; extra: [(k, D1, D2, cJ, cK)] density pairs
        added to output k (D1, D2 device [nao][nao])."""
        import torch
        _check_dev(X, self.device, "X")
        _check_dev(Y, self.device, "Y")
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        if out is None:
            out = torch.empty((sel.size, self.natm, 3), dtype=torch.float64, device=self.device)
        _check_dev(out, self.device, "grad")
        ne, ea = _extra_array(extra, self.device, self.nao)
        self._chk(self.lib.ris_grad_contract(self.h, X.shape[0], _ptr(X), _ptr(Y), sel.size,
                                             sel.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ne, ea, _ptr(out)))
        return out

    def nac_contract(self, X, Y, pairs, omega=None, out=None, allow_degenerate=False, extra=None):
        import torch
        _check_dev(X, self.device, "X")
        _check_dev(Y, self.device, "Y")
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        if out is None:
            out = torch.empty((pairs.shape[0], self.natm, 3), dtype=torch.float64, device=self.device)
        _check_dev(out, self.device, "nac")
        om = None
        if omega is not None:
            om = np.ascontiguousarray(omega, dtype=np.float64)
        ne, ea = _extra_array(extra, self.device, self.nao)
        st = self.lib.ris_nac_contract(self.h, X.shape[0], _ptr(X), _ptr(Y), pairs.shape[0],
                                       pairs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ne, ea,
                                       om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if om is not None else None,
                                       _ptr(out))
        if st == 5 and allow_degenerate:
            return out
        self._chk(st)
        return out


def _grad_nac_impl(self, X, Y, sel, pairs, omega=None, grad=None, nac=None, allow_degenerate=False, extra=None):
    import torch
    _check_dev(X, self.device, "X")
    _check_dev(Y, self.device, "Y")
    sel = np.ascontiguousarray(sel, dtype=np.int32).reshape(-1)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    if grad is None:
        grad = torch.empty((sel.size, self.natm, 3), dtype=torch.float64, device=self.device)
    if nac is None:
        nac = torch.empty((pairs.shape[0], self.natm, 3), dtype=torch.float64, device=self.device)
    _check_dev(grad, self.device, "grad")
    _check_dev(nac, self.device, "nac")
    om = None if omega is None else np.ascontiguousarray(omega, dtype=np.float64)
    ip = ctypes.POINTER(ctypes.c_int)
    ne, ea = _extra_array(extra, self.device, self.nao)
    st = self.lib.ris_grad_nac_contract(
        self.h, X.shape[0], _ptr(X), _ptr(Y), sel.size, sel.ctypes.data_as(ip), _ptr(grad), pairs.shape[0],
        pairs.ctypes.data_as(ip), om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if om is not None else None,
        _ptr(nac), ne, ea)
    if not (st == 5 and allow_degenerate):
        self._chk(st)
    return grad, nac


RisContext.grad_nac_contract = _grad_nac_impl


def solve_problem(ctx: RisContext, prob, radius_bohr, outputs, theta=0.2, j_p_on_heavy=True, alpha_J=2.0,
                  c_x=0.25, dbg=False):
    """Convenience driver for a molgen.Problem: aux_build -> int3c -> grad/nac.
    outputs: list of (I, J); I == J are gradients, I != J NAC numerators.
    Returns a torch tensor [nout][natm][3] on the device."""
    import torch
    dev = ctx.device
    m = prob.mol
    ctx.aux_build(m.Z, m.xyz, m.shell_atom, m.shell_l, m.shell_exp, radius_bohr, theta, j_p_on_heavy)
    C = torch.as_tensor(prob.C, device=dev).contiguous()
    eps = torch.as_tensor(prob.eps, device=dev).contiguous()
    X = torch.as_tensor(prob.X, device=dev).contiguous()
    Y = None if prob.Y is None else torch.as_tensor(prob.Y, device=dev).contiguous()
    dbg_t = torch.empty((ctx.nJ, m.nao, m.nao), dtype=torch.float64, device=dev) if dbg else None
    ctx.int3c(C, eps, prob.nocc, alpha_J, c_x, dbg=dbg_t)
    out = torch.empty((len(outputs), m.natm, 3), dtype=torch.float64, device=dev)
    grads = [k for k, (I, J) in enumerate(outputs) if I == J]
    nacs = [k for k, (I, J) in enumerate(outputs) if I != J]
    if grads:
        g = ctx.grad_contract(X, Y, [outputs[k][0] for k in grads])
        out[grads] = g
    if nacs:
        n = ctx.nac_contract(X, Y, [outputs[k] for k in nacs])
        out[nacs] = n
    return (out, dbg_t) if dbg else out

"""Python binding of the C-ABI library libvdwxc_gpu.so (include/vdwxc_gpu.h).

Argument marshalling only: every step of the evaluation runs in the library's HIP kernels.  torch
provides device memory and the stream.  The binding refuses to run without the built library
(there is no CPU fallback).

    f = Functional(grid, cell, flavour="DF1", precision="fp64", table=kernel_table)
    E, dedn, dedsigma = f.calculate(n, sigma)          # paper form: partial derivatives
    E, v = f.potential(n, grad=None)                   # v = dE/dn - div(2 dE/dsigma grad n)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libvdwxc_gpu.so")

OK, EINVAL, ENOMEM, EDEVICE, ETABLE, ESTATE = range(6)
DF1, DF2 = 1, 2
FP64, FP32_MIXED = 0, 1
INIT_NO_WORKSPACE = 1
FLAVOURS = {"DF1": DF1, "DF2": DF2, "vdW-DF1": DF1, "vdW-DF2": DF2}
PRECISIONS = {"fp64": FP64, "fp32": FP32_MIXED, "fp32_mixed": FP32_MIXED}

# every entry point the header declares, with its ctypes signature
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_h = ctypes.c_void_p
SIGNATURES = {
    "vdwxc_init": (ctypes.c_int, [ctypes.POINTER(_h), _ip, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_void_p]),
    "vdwxc_init_table": (ctypes.c_int, [ctypes.POINTER(_h), _ip, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                        ctypes.c_int, ctypes.c_double, _dp, ctypes.c_void_p]),
    "vdwxc_init_table_ex": (ctypes.c_int, [ctypes.POINTER(_h), _ip, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                           ctypes.c_int, ctypes.c_double, _dp, ctypes.c_void_p, ctypes.c_uint]),
    "vdwxc_set_workspace": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_size_t]),
    "vdwxc_calculate": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _dp]),
    "vdwxc_calculate_async": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]),
    "vdwxc_calculate_potential": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, _dp]),
    "vdwxc_calculate_potential_async": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                       ctypes.c_void_p]),
    "vdwxc_calculate_lda_async": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "vdwxc_calculate_spin": (ctypes.c_int, [_h] + [ctypes.c_void_p] * 8 + [_dp]),
    "vdwxc_calculate_spin_async": (ctypes.c_int, [_h] + [ctypes.c_void_p] * 9),
    "vdwxc_calculate_spin_potential": (ctypes.c_int, [_h] + [ctypes.c_void_p] * 6 + [_dp]),
    "vdwxc_calculate_spin_potential_async": (ctypes.c_int, [_h] + [ctypes.c_void_p] * 7),
    "vdwxc_calculate_potential_noalloc": (ctypes.c_int, [_h, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                         ctypes.c_void_p]),
    "vdwxc_workspace_bytes": (ctypes.c_size_t, [_ip, ctypes.c_int]),
    "vdwxc_workspace_bytes_m": (ctypes.c_size_t, [_ip, ctypes.c_int, ctypes.c_int]),
    "vdwxc_set_stream": (ctypes.c_int, [_h, ctypes.c_void_p]),
    "vdwxc_print": (ctypes.c_int, [_h]),
    "vdwxc_finalize": (ctypes.c_int, [ctypes.POINTER(_h)]),
    "vdwxc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "vdwxc_last_error": (ctypes.c_char_p, [_h]),
    "vdwxc_version": (ctypes.c_char_p, []),
    "vdwxc_enable_timing": (ctypes.c_int, [_h, ctypes.c_int]),
    "vdwxc_read_timing": (ctypes.c_int, [_h, _dp, ctypes.POINTER(ctypes.c_longlong)]),
    "vdwxc_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
}
NUM_STAGES = 13

_lib = None


class VdwxcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vdwxc status {status}: {message}")
        self.status = status


def library_available() -> bool:
    return os.path.exists(LIB_PATH)


def lib():
    """Load libvdwxc_gpu.so (once); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1703_06999_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int, handle=None):
    if status != OK:
        L = lib()
        msg = L.vdwxc_last_error(handle).decode() if handle is not None else L.vdwxc_last_error(None).decode()
        raise VdwxcError(status, f"{L.vdwxc_strerror(status).decode()}: {msg}")


def workspace_bytes(grid, precision="fp64", nq: int = 20) -> int:
    """Device bytes of a handle's work buffers (vdwxc_workspace_bytes_m)."""
    g = (ctypes.c_int * 3)(*[int(x) for x in grid])
    return int(lib().vdwxc_workspace_bytes_m(g, PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                                             int(nq)))


def _cell_array(cell):
    c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(9))
    return (ctypes.c_double * 9)(*c.tolist())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Functional:
    """A library handle for one grid, cell, flavour, precision and kernel table."""

    def __init__(self, grid, cell, flavour="DF1", precision="fp64", table=None, stream=None, table_path=None,
                 own_workspace: bool = True):
        import torch
        self.grid = tuple(int(x) for x in grid)
        self.cell = np.asarray(cell, dtype=np.float64).reshape(3, 3)
        self.precision = precision
        self.flavour = flavour
        self.omega = float(np.linalg.det(self.cell))
        self.npoints = int(np.prod(self.grid))
        self.dV = self.omega / self.npoints
        self._stream = stream
        self._h = ctypes.c_void_p()
        L = lib()
        g = (ctypes.c_int * 3)(*self.grid)
        fl = FLAVOURS[flavour] if isinstance(flavour, str) else int(flavour)
        pr = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if table_path is not None and not own_workspace:
            raise ValueError("a handle without its own work memory takes the kernel table as arrays (table=...)")
        with torch.cuda.device(torch.cuda.current_device()):
            sh = _stream_handle(stream)
            if table_path is not None:
                st = L.vdwxc_init(ctypes.byref(self._h), g, _cell_array(self.cell), fl, pr,
                                  str(table_path).encode(), sh)
            else:
                q = np.ascontiguousarray(table.qmesh, dtype=np.float64)
                t = np.ascontiguousarray(table.table, dtype=np.float64)
                st = L.vdwxc_init_table_ex(ctypes.byref(self._h), g, _cell_array(self.cell), fl, pr, int(q.shape[0]),
                                           q.ctypes.data_as(_dp), int(t.shape[0]), float(table.kmax),
                                           t.ctypes.data_as(_dp), sh, 0 if own_workspace else INIT_NO_WORKSPACE)
        _check(st)
        self.nq = int(table.nq) if table is not None else None

    # -- helpers -------------------------------------------------------------------------------
    def _field(self, x, name, comps=None):
        import torch
        shape = self.grid if comps is None else (comps,) + self.grid
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if x.dtype != torch.float64 or tuple(x.shape) != shape or not x.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape}")
        return ctypes.c_void_p(x.data_ptr())

    def _sync_stream(self):
        L = lib()
        _check(L.vdwxc_set_stream(self._h, _stream_handle(self._stream)), self._h)

    # -- entry points ----------------------------------------------------------------------------
    def calculate(self, n, sigma, dedn=None, dedsigma=None):
        """(E, dedn, dedsigma): paper Sec. 3 steps 1-5 and eqs. dedn, dedsigma."""
        import torch
        dedn = torch.empty_like(n) if dedn is None else dedn
        dedsigma = torch.empty_like(n) if dedsigma is None else dedsigma
        e = ctypes.c_double(0.0)
        self._sync_stream()
        st = lib().vdwxc_calculate(self._h, self._field(n, "n"), self._field(sigma, "sigma"),
                                   self._field(dedn, "dedn"), self._field(dedsigma, "dedsigma"), ctypes.byref(e))
        _check(st, self._h)
        return e.value, dedn, dedsigma

    def calculate_async(self, n, sigma, dedn, dedsigma, energy):
        """Enqueue the partials evaluation; energy is a 1-element float64 device tensor."""
        self._sync_stream()
        st = lib().vdwxc_calculate_async(self._h, self._field(n, "n"), self._field(sigma, "sigma"),
                                         self._field(dedn, "dedn"), self._field(dedsigma, "dedsigma"),
                                         ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def potential(self, n, grad=None, v=None):
        """(E, v) with v = dE/dn - div(2 dE/dsigma grad n); grad None = spectral gradient."""
        import torch
        v = torch.empty_like(n) if v is None else v
        e = ctypes.c_double(0.0)
        gp = self._field(grad, "grad", 3) if grad is not None else ctypes.c_void_p(0)
        self._sync_stream()
        st = lib().vdwxc_calculate_potential(self._h, self._field(n, "n"), gp, self._field(v, "v"), ctypes.byref(e))
        _check(st, self._h)
        return e.value, v

    def potential_async(self, n, grad, v, energy):
        """Enqueue the potential evaluation on the handle's stream; nothing is synchronised."""
        gp = self._field(grad, "grad", 3) if grad is not None else ctypes.c_void_p(0)
        self._sync_stream()
        st = lib().vdwxc_calculate_potential_async(self._h, self._field(n, "n"), gp, self._field(v, "v"),
                                                   ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def potential_noalloc(self, n, grad, v, energy):
        """As potential_async, with the work buffers in the library's static array (allocates
        nothing; calls on one device must not overlap; grids up to 128 MiB of work memory)."""
        gp = self._field(grad, "grad", 3) if grad is not None else ctypes.c_void_p(0)
        self._sync_stream()
        st = lib().vdwxc_calculate_potential_noalloc(self._h, self._field(n, "n"), gp, self._field(v, "v"),
                                                     ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def lda_async(self, n, v, energy):
        """Enqueue the PW92 LDA correlation: E_c^LDA into the 1-element float64 device tensor
        `energy`, v_c^LDA into `v`."""
        self._sync_stream()
        st = lib().vdwxc_calculate_lda_async(self._h, self._field(n, "n"), self._field(v, "v"),
                                             ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def lda(self, n, v=None):
        """(E_c^LDA, v_c^LDA) of the appendix's PW92 correlation; synchronises the stream."""
        import torch
        v = torch.empty_like(n) if v is None else v
        e = torch.empty(1, dtype=torch.float64, device=n.device)
        self.lda_async(n, v, e)
        torch.cuda.synchronize(n.device)
        return float(e.item()), v

    def spin_async(self, n_up, n_dn, sigma_uu, sigma_dd, outs, energy):
        """Enqueue the spin-polarised partials evaluation: outs = (dedn_up, dedn_dn, dedsigma_uu,
        dedsigma_dd) device tensors (distinct from the inputs), energy a 1-element float64 tensor."""
        self._sync_stream()
        ins = [self._field(a, k) for a, k in ((n_up, "n_up"), (n_dn, "n_dn"), (sigma_uu, "sigma_uu"),
                                              (sigma_dd, "sigma_dd"))]
        os_ = [self._field(a, k) for a, k in zip(outs, ("dedn_up", "dedn_dn", "dedsigma_uu", "dedsigma_dd"))]
        st = lib().vdwxc_calculate_spin_async(self._h, *ins, *os_, ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def spin(self, n_up, n_dn, sigma_uu, sigma_dd):
        """(E, dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd) of the spin-polarised functional
        (vdwxc_calculate_spin); synchronises the stream."""
        import torch
        outs = [torch.empty_like(n_up) for _ in range(4)]
        e = ctypes.c_double(0.0)
        self._sync_stream()
        ins = [self._field(a, k) for a, k in ((n_up, "n_up"), (n_dn, "n_dn"), (sigma_uu, "sigma_uu"),
                                              (sigma_dd, "sigma_dd"))]
        os_ = [self._field(a, k) for a, k in zip(outs, ("dedn_up", "dedn_dn", "dedsigma_uu", "dedsigma_dd"))]
        st = lib().vdwxc_calculate_spin(self._h, *ins, *os_, ctypes.byref(e))
        _check(st, self._h)
        return (e.value, *outs)

    def spin_potential_async(self, n_up, n_dn, grad_up, grad_dn, v_up, v_dn, energy):
        """Enqueue the spin-polarised potentials (vdwxc_calculate_spin_potential_async)."""
        self._sync_stream()
        st = lib().vdwxc_calculate_spin_potential_async(
            self._h, self._field(n_up, "n_up"), self._field(n_dn, "n_dn"), self._field(grad_up, "grad_up", 3),
            self._field(grad_dn, "grad_dn", 3), self._field(v_up, "v_up"), self._field(v_dn, "v_dn"),
            ctypes.c_void_p(energy.data_ptr()))
        _check(st, self._h)

    def spin_potential(self, n_up, n_dn, grad_up, grad_dn):
        """(E, v_up, v_dn) of the spin-polarised functional; synchronises the stream."""
        import torch
        v_up, v_dn = torch.empty_like(n_up), torch.empty_like(n_up)
        e = ctypes.c_double(0.0)
        self._sync_stream()
        st = lib().vdwxc_calculate_spin_potential(
            self._h, self._field(n_up, "n_up"), self._field(n_dn, "n_dn"), self._field(grad_up, "grad_up", 3),
            self._field(grad_dn, "grad_dn", 3), self._field(v_up, "v_up"), self._field(v_dn, "v_dn"), ctypes.byref(e))
        _check(st, self._h)
        return e.value, v_up, v_dn

    def set_workspace(self, buf):
        """Run later calls in `buf` (a CUDA tensor of at least workspace_bytes(grid, precision, nq)
        bytes, kept alive by the caller while work enqueued with it is pending); None returns the
        handle to its own work memory."""
        self._sync_stream()
        if buf is None:
            st = lib().vdwxc_set_workspace(self._h, None, 0)
        else:
            if not buf.is_cuda or not buf.is_contiguous():
                raise ValueError("workspace must be a contiguous CUDA tensor")
            st = lib().vdwxc_set_workspace(self._h, ctypes.c_void_p(buf.data_ptr()),
                                           buf.numel() * buf.element_size())
        _check(st, self._h)

    def enable_timing(self, enable: bool = True):
        """Record HIP events around every kernel launch of this handle (see read_timing)."""
        _check(lib().vdwxc_enable_timing(self._h, int(bool(enable))), self._h)

    def read_timing(self):
        """{stage name: (total ms, launches)} since the last enable/read; synchronises."""
        ms = (ctypes.c_double * NUM_STAGES)()
        cnt = (ctypes.c_longlong * NUM_STAGES)()
        _check(lib().vdwxc_read_timing(self._h, ms, cnt), self._h)
        L = lib()
        return {L.vdwxc_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NUM_STAGES) if cnt[i] > 0}

    def set_stream(self, stream):
        self._stream = stream
        self._sync_stream()

    def print(self):
        _check(lib().vdwxc_print(self._h), self._h)

    def close(self):
        if self._h is not None and self._h.value:
            lib().vdwxc_finalize(ctypes.byref(self._h))
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

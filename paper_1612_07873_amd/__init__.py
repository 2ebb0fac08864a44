"""MI355X-native adaptive-multigrid Wilson-clover kernels (gfx950 HIP).

Python side of the qmg C ABI: thin wrappers that pass torch device tensors'
data pointers and the current HIP stream to libqmg.so.  Every step runs in
the library's kernels; if the library is missing, these calls raise.
"""
import ctypes
import json
import os

import numpy as np
import torch

from . import _lib
from ._lib import PREC, QmgError, lib

__all__ = ['BiCGStab', 'sync', 'stream_read', 'tune_cache_save', 'tune_cache_load', 'tune_cache_clear', 'apply_mrhs_multi', 'PTC', 'quantize_sites', 'dequantize_sites', 'CoarseOp', 'FineOp', 'Transfer', 'build_coarse_op', 'Multigrid', 'QmgError', 'lib', 'stream_ptr', 'PREC']

_CDTYPE = {'c128': torch.complex128, 'c64': torch.complex64}
_VECDTYPE = {'c128': torch.complex128, 'c64': torch.complex64, 'h16': torch.complex64, 'b16': torch.complex64}


def stream_read(buf, sink):
    """Read the device tensor `buf` once with the library's read-stream kernel (qmg_stream_read);
    sink: int32 device tensor of at least 16 x (compute units) words."""
    _lib.call('qmg_stream_read', ctypes.c_void_p(buf.data_ptr()), int(buf.numel() * buf.element_size()),
              ctypes.c_void_p(sink.data_ptr()), int(sink.numel()), stream_ptr())


def sync():
    """Wait for the current stream (qmg_sync); raises QmgError with QMG_ERR_NONFINITE if a
    16-bit encoder met a NaN or Inf input since the last report."""
    _lib.call('qmg_sync', stream_ptr())


def tune_cache_save(path):
    """Write the autotuner's in-process choices to the text file `path`
    (qmg_tune_cache_save); returns the number of entries."""
    n = ctypes.c_int(0)
    _lib.call('qmg_tune_cache_save', os.fsencode(path), ctypes.byref(n))
    return n.value


def tune_cache_load(path):
    """Merge the entries of a file written by tune_cache_save on this device
    architecture and HIP runtime into the autotuner's cache
    (qmg_tune_cache_load); returns the number of entries read."""
    n = ctypes.c_int(0)
    _lib.call('qmg_tune_cache_load', os.fsencode(path), ctypes.byref(n))
    return n.value


def tune_cache_clear():
    """Empty the autotuner's in-process cache (qmg_tune_cache_clear)."""
    _lib.call('qmg_tune_cache_clear')


def stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, shape, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError('%s must be a device tensor' % what)
    if t.dtype != dtype:
        raise TypeError('%s must be %s, got %s' % (what, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError('%s must have shape %s, got %s' % (what, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError('%s must be contiguous' % what)
    return ctypes.c_void_p(t.data_ptr())


def _nrhs(t, tail, what):
    """Right-hand sides of a field given as tail (one) or [nrhs] + tail (several)."""
    if isinstance(t, torch.Tensor) and t.dim() == len(tail) + 1:
        return int(t.shape[0]), (int(t.shape[0]),) + tuple(tail)
    return 1, tuple(tail)


def _vol(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


class CoarseOp:
    """Coarse operator of Eq. (3) held by the library (see qmg_coarse_op_create)."""

    def __init__(self, dims, X, Y, storage='c128', _handle=None, _N=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = _vol(self.dims)
        self.storage = storage
        self.dtype = _VECDTYPE[storage]
        if _handle is not None:
            self.N = int(_N)
            self._h = _handle
            return
        self.N = int(X.shape[-1])
        h = ctypes.c_void_p()
        _lib.call('qmg_coarse_op_create', _lib.c_dims(*self.dims), self.N,
                  _dev_ptr(X, torch.complex128, (self.V, self.N, self.N), 'X'),
                  _dev_ptr(Y, torch.complex128, (8, self.V, self.N, self.N), 'Y'),
                  PREC[storage], stream_ptr(), ctypes.byref(h))
        self._h = h

    def apply(self, u, out=None):
        """Eq. (3) on u [V][N] or, for several right-hand sides, [nrhs][V][N]."""
        if out is None:
            out = torch.empty_like(u)
        vp = self.storage if self.storage in ('c128', 'c64') else 'c64'
        m, shape = _nrhs(u, (self.V, self.N), 'in')
        _lib.call('qmg_coarse_dslash', self._h,
                  _dev_ptr(u, self.dtype, shape, 'in'),
                  _dev_ptr(out, self.dtype, shape, 'out'),
                  m, PREC[vp], stream_ptr())
        return out

    def apply_mrhs(self, u16, uscale, out=None):
        """Multi-RHS: u16 int32 [V][nrhs][N] packed 16-bit pairs, uscale float32 [V][nrhs];
        returns complex64 [V][nrhs][N]."""
        V, nrhs, N = u16.shape
        if out is None:
            out = torch.empty((V, nrhs, N), dtype=torch.complex64, device=u16.device)
        _lib.call('qmg_coarse_dslash_mrhs', self._h, _dev_ptr(u16, torch.int32, (self.V, nrhs, self.N), 'in'),
                  _dev_ptr(uscale, torch.float32, (self.V, nrhs), 'in_scale'),
                  _dev_ptr(out, torch.complex64, (self.V, nrhs, self.N), 'out'), int(nrhs), stream_ptr())
        return out

    def apply_mrhs_c64(self, u, out=None):
        """Matrix-core batch from complex64 fields: u [nrhs][V][N] -> [nrhs][V][N] (16-bit operators)."""
        nrhs = int(u.shape[0])
        if out is None:
            out = torch.empty_like(u)
        _lib.call('qmg_coarse_dslash_mrhs_c64', self._h, _dev_ptr(u, torch.complex64, (nrhs, self.V, self.N), 'in'),
                  _dev_ptr(out, torch.complex64, (nrhs, self.V, self.N), 'out'), nrhs, stream_ptr())
        return out

    def set_mrhs_tiles(self, nrhs, tiles):
        _lib.call('qmg_coarse_op_set_mrhs_tiles', self._h, int(nrhs), int(tiles))

    def mrhs_tiles(self, nrhs):
        t = ctypes.c_int()
        _lib.call('qmg_coarse_op_get_mrhs_tiles', self._h, int(nrhs), ctypes.byref(t))
        return t.value

    def apply_scaled(self, u16, uscale, out16=None, oscale=None, vprec=None):
        """16-bit vectors: u16 int32 tensor [V][N] (packed pairs), uscale float32 [V]."""
        vprec = vprec or self.storage
        if out16 is None:
            out16 = torch.empty_like(u16)
        if oscale is None:
            oscale = torch.empty_like(uscale)
        _lib.call('qmg_coarse_dslash_scaled', self._h, _dev_ptr(u16, torch.int32, (self.V, self.N), 'in'),
                  _dev_ptr(uscale, torch.float32, (self.V,), 'in_scale'),
                  _dev_ptr(out16, torch.int32, (self.V, self.N), 'out'),
                  _dev_ptr(oscale, torch.float32, (self.V,), 'out_scale'), PREC[vprec], stream_ptr())
        return out16, oscale

    # red-black form (Sec. 3.3): half-lattice fields [V/2][N] of the even sites
    def prepare_schur(self):
        _lib.call('qmg_coarse_op_prepare_schur', self._h, stream_ptr())

    def _vp(self):
        return self.storage if self.storage in ('c128', 'c64') else 'c64'

    def schur(self, ue, out=None):
        """S u_e = (X_ee - Y_eo X_oo^-1 Y_oe) u_e for u_e [V/2][N] or [nrhs][V/2][N]."""
        if out is None:
            out = torch.empty_like(ue)
        m, shape = _nrhs(ue, (self.V // 2, self.N), 'in_e')
        _lib.call('qmg_coarse_dslash_schur', self._h, _dev_ptr(ue, self.dtype, shape, 'in_e'),
                  _dev_ptr(out, self.dtype, shape, 'out_e'), m, PREC[self._vp()], stream_ptr())
        return out

    def schur_source(self, b, out=None):
        """b_e - Y_eo X_oo^-1 b_o for whole-lattice b [V][N] (or [nrhs][V][N])."""
        m, shape = _nrhs(b, (self.V, self.N), 'b')
        hshape = shape[:-2] + (self.V // 2, self.N)
        if out is None:
            out = torch.empty(hshape, dtype=b.dtype, device=b.device)
        _lib.call('qmg_coarse_schur_source', self._h, _dev_ptr(b, self.dtype, shape, 'b'),
                  _dev_ptr(out, self.dtype, hshape, 'bhat_e'), m, PREC[self._vp()], stream_ptr())
        return out

    def schur_reconstruct(self, xe, b, out=None):
        """Whole-lattice x: x_e given, x_o = X_oo^-1 (b_o - Y_oe x_e)."""
        m, shape = _nrhs(b, (self.V, self.N), 'b')
        hshape = shape[:-2] + (self.V // 2, self.N)
        if out is None:
            out = torch.empty_like(b)
        _lib.call('qmg_coarse_schur_reconstruct', self._h, _dev_ptr(xe, self.dtype, hshape, 'x_e'),
                  _dev_ptr(b, self.dtype, shape, 'b'), _dev_ptr(out, self.dtype, shape, 'x'), m,
                  PREC[self._vp()], stream_ptr())
        return out

    def export(self):
        dev = torch.device('cuda')
        X = torch.empty((self.V, self.N, self.N), dtype=torch.complex128, device=dev)
        Y = torch.empty((8, self.V, self.N, self.N), dtype=torch.complex128, device=dev)
        _lib.call('qmg_coarse_op_export', self._h, ctypes.c_void_p(X.data_ptr()),
                  ctypes.c_void_p(Y.data_ptr()), stream_ptr())
        return X, Y

    def tune(self, u, out, cold=False, u16=None, uscale=None, o16=None, oscale=None):
        """Autotune the single-RHS launch on these fields; returns the best time in ms."""
        ms = ctypes.c_float()
        if u16 is None:
            vp = self.storage if self.storage in ('c128', 'c64') else 'c64'
            _lib.call('qmg_coarse_op_tune', self._h, _dev_ptr(u, self.dtype, (self.V, self.N), 'in'), None,
                      _dev_ptr(out, self.dtype, (self.V, self.N), 'out'), None, PREC[vp], int(bool(cold)),
                      stream_ptr(), ctypes.byref(ms))
        else:
            _lib.call('qmg_coarse_op_tune', self._h, ctypes.c_void_p(u16.data_ptr()), ctypes.c_void_p(uscale.data_ptr()),
                      ctypes.c_void_p(o16.data_ptr()), ctypes.c_void_p(oscale.data_ptr()), PREC[self.storage],
                      int(bool(cold)), stream_ptr(), ctypes.byref(ms))
        return ms.value

    def tune_mrhs(self, u16, uscale, out, cold=False):
        V, nrhs, N = u16.shape
        ms = ctypes.c_float()
        _lib.call('qmg_coarse_op_tune_mrhs', self._h, _dev_ptr(u16, torch.int32, (self.V, nrhs, self.N), 'in'),
                  _dev_ptr(uscale, torch.float32, (self.V, nrhs), 'in_scale'),
                  _dev_ptr(out, torch.complex64, (self.V, nrhs, self.N), 'out'), int(nrhs), int(bool(cold)),
                  stream_ptr(), ctypes.byref(ms))
        return ms.value

    def prefetch(self):
        p = ctypes.c_int()
        _lib.call('qmg_coarse_op_get_prefetch', self._h, ctypes.byref(p))
        return p.value

    def set_launch(self, rows=0, split=0):
        _lib.call('qmg_coarse_op_set_launch', self._h, int(rows), int(split))

    def launch(self):
        r, s = ctypes.c_int(), ctypes.c_int()
        _lib.call('qmg_coarse_op_get_launch', self._h, ctypes.byref(r), ctypes.byref(s))
        return r.value, s.value

    @property
    def chunks_per_row(self):
        return 9 * self.N // (1 if self.storage == 'c128' else 2)

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None and not getattr(self, '_borrowed', False):
            _lib._lib.qmg_coarse_op_destroy(h)
            self._h = None


class FineOp:
    """Wilson-clover operator of Eq. (2) held by the library (qmg_fine_op_create).
    storage 'h16' / 'b16' keeps links and clover in 16 bits; apply() then takes
    complex64 vectors and apply_scaled() 16-bit vectors with per-site scales."""

    def __init__(self, dims, gauge, m0, csw=1.0, antiperiodic_t=True, storage='c128', link_reals=18):
        self.dims = tuple(int(d) for d in dims)
        self.V = _vol(self.dims)
        self.storage = storage
        self.dtype = _VECDTYPE[storage]
        self.m0, self.csw = float(m0), float(csw)
        self.link_reals = int(link_reals)
        h = ctypes.c_void_p()
        _lib.call('qmg_fine_op_create_ex', _lib.c_dims(*self.dims),
                  _dev_ptr(gauge, torch.complex128, (4, self.V, 3, 3), 'gauge'),
                  self.m0, self.csw, int(bool(antiperiodic_t)), PREC[storage], self.link_reals, stream_ptr(),
                  ctypes.byref(h))
        self._h = h

    def sap(self, r, block, iters, out=None):
        """One Schwarz alternating procedure sweep x = SAP(r) (qmg_wilson_clover_sap);
        r complex64 [V][4][3] or [nrhs][V][4][3]."""
        if out is None:
            out = torch.empty_like(r)
        m, shape = _nrhs(r, (self.V, 4, 3), 'r')
        _lib.call('qmg_wilson_clover_sap', self._h, _lib.c_dims(*block), int(iters),
                  _dev_ptr(r, torch.complex64, shape, 'r'), _dev_ptr(out, torch.complex64, shape, 'x'), m,
                  stream_ptr())
        return out

    def apply(self, psi, out=None):
        """Eq. (2) on psi [V][4][3] or, for several fields, [nrhs][V][4][3]."""
        if out is None:
            out = torch.empty_like(psi)
        vp = self.storage if self.storage in ('c128', 'c64') else 'c64'
        m, shape = _nrhs(psi, (self.V, 4, 3), 'in')
        _lib.call('qmg_wilson_clover_dslash', self._h,
                  _dev_ptr(psi, self.dtype, shape, 'in'),
                  _dev_ptr(out, self.dtype, shape, 'out'), m, PREC[vp], stream_ptr())
        return out

    def apply_scaled(self, u16, uscale, out16=None, oscale=None, vprec=None):
        """16-bit spinors: u16 int32 [V][12] (packed pairs), uscale float32 [V]."""
        vprec = vprec or self.storage
        if out16 is None:
            out16 = torch.empty_like(u16)
        if oscale is None:
            oscale = torch.empty_like(uscale)
        _lib.call('qmg_wilson_clover_dslash_scaled', self._h, _dev_ptr(u16, torch.int32, (self.V, 12), 'in'),
                  _dev_ptr(uscale, torch.float32, (self.V,), 'in_scale'),
                  _dev_ptr(out16, torch.int32, (self.V, 12), 'out'),
                  _dev_ptr(oscale, torch.float32, (self.V,), 'out_scale'), PREC[vprec], stream_ptr())
        return out16, oscale

    # red-black form (Sec. 3.3): half-lattice fields [V/2][4][3] of the even sites
    def _vp(self):
        return self.storage if self.storage in ('c128', 'c64') else 'c64'

    def schur_scaled(self, u16, uscale, out16=None, oscale=None):
        """S on 16-bit half-lattice spinors: u16 int32 [V/2][12] (or [nrhs][V/2][12]) FP16
        pairs, uscale float32 [V/2] (or [nrhs][V/2]) (qmg_wilson_clover_schur_scaled)."""
        if out16 is None:
            out16 = torch.empty_like(u16)
        if oscale is None:
            oscale = torch.empty_like(uscale)
        m, shape = _nrhs(u16, (self.V // 2, 12), 'in_e')
        _lib.call('qmg_wilson_clover_schur_scaled', self._h, _dev_ptr(u16, torch.int32, shape, 'in_e'),
                  _dev_ptr(uscale, torch.float32, shape[:-1], 'in_scale'), _dev_ptr(out16, torch.int32, shape, 'out_e'),
                  _dev_ptr(oscale, torch.float32, shape[:-1], 'out_scale'), m, stream_ptr())
        return out16, oscale

    def schur(self, pe, out=None):
        """S p_e = (C_ee - D_eo C_oo^-1 D_oe) p_e, C = 4 + m0 + A, D the hops of Eq. (2)."""
        if out is None:
            out = torch.empty_like(pe)
        m, shape = _nrhs(pe, (self.V // 2, 4, 3), 'in_e')
        _lib.call('qmg_wilson_clover_schur', self._h, _dev_ptr(pe, self.dtype, shape, 'in_e'),
                  _dev_ptr(out, self.dtype, shape, 'out_e'), m, PREC[self._vp()], stream_ptr())
        return out

    def schur_source(self, b, out=None):
        """b_e - D_eo C_oo^-1 b_o for whole-lattice b [V][4][3] (or [nrhs][V][4][3])."""
        m, shape = _nrhs(b, (self.V, 4, 3), 'b')
        hshape = shape[:-3] + (self.V // 2, 4, 3)
        if out is None:
            out = torch.empty(hshape, dtype=b.dtype, device=b.device)
        _lib.call('qmg_wilson_clover_schur_source', self._h, _dev_ptr(b, self.dtype, shape, 'b'),
                  _dev_ptr(out, self.dtype, hshape, 'bhat_e'), m, PREC[self._vp()], stream_ptr())
        return out

    def schur_reconstruct(self, xe, b, out=None):
        """Whole-lattice x: x_e given, x_o = C_oo^-1 (b_o - D_oe x_e)."""
        m, shape = _nrhs(b, (self.V, 4, 3), 'b')
        hshape = shape[:-3] + (self.V // 2, 4, 3)
        if out is None:
            out = torch.empty_like(b)
        _lib.call('qmg_wilson_clover_schur_reconstruct', self._h, _dev_ptr(xe, self.dtype, hshape, 'x_e'),
                  _dev_ptr(b, self.dtype, shape, 'b'), _dev_ptr(out, self.dtype, shape, 'x'), m,
                  PREC[self._vp()], stream_ptr())
        return out

    def clover(self):
        A = torch.empty((self.V, 12, 12), dtype=torch.complex128, device='cuda')
        _lib.call('qmg_fine_op_export_clover', self._h, ctypes.c_void_p(A.data_ptr()), stream_ptr())
        return A

    def links(self):
        """The links as stored (complex128 [4][V][3][3], time sign removed)."""
        G = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device='cuda')
        _lib.call('qmg_fine_op_export_links', self._h, ctypes.c_void_p(G.data_ptr()), stream_ptr())
        return G

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.qmg_fine_op_destroy(h)
            self._h = None


class Transfer:
    """Prolongator / restrictor built from near-null vectors (qmg_transfer_create)."""

    def __init__(self, fine_dims, fine_dof, block, nullvecs, storage='c128'):
        self.fine_dims = tuple(int(d) for d in fine_dims)
        self.V = _vol(self.fine_dims)
        self.dof = int(fine_dof)
        self.block = tuple(int(b) for b in block)
        self.nvec = int(nullvecs.shape[0])
        self.storage = storage
        h = ctypes.c_void_p()
        _lib.call('qmg_transfer_create', _lib.c_dims(*self.fine_dims), self.dof, _lib.c_dims(*self.block),
                  self.nvec, _dev_ptr(nullvecs, torch.complex128, (self.nvec, self.V, self.dof), 'nullvecs'),
                  PREC[storage], stream_ptr(), ctypes.byref(h))
        self._h = h
        cd = _lib.c_dims()
        n = ctypes.c_int()
        _lib.call('qmg_transfer_coarse_dims', h, cd, ctypes.byref(n))
        self.coarse_dims = tuple(cd)
        self.Vc = _vol(self.coarse_dims)
        self.N = n.value

    @classmethod
    def from_basis(cls, fine_dims, fine_dof, block, basis, storage='c128'):
        """Transfer from a finished block-orthonormal basis, complex128 [V][fine_dof][nvec] as
        basis() returns it (qmg_transfer_import: no orthonormalisation)."""
        t = cls.__new__(cls)
        t.fine_dims = tuple(int(d) for d in fine_dims)
        t.V = _vol(t.fine_dims)
        t.dof = int(fine_dof)
        t.block = tuple(int(b) for b in block)
        t.nvec = int(basis.shape[-1])
        t.storage = storage
        h = ctypes.c_void_p()
        _lib.call('qmg_transfer_import', _lib.c_dims(*t.fine_dims), t.dof, _lib.c_dims(*t.block), t.nvec,
                  _dev_ptr(basis, torch.complex128, (t.V, t.dof, t.nvec), 'basis'), PREC[storage], stream_ptr(),
                  ctypes.byref(h))
        t._h = h
        cd = _lib.c_dims()
        n = ctypes.c_int()
        _lib.call('qmg_transfer_coarse_dims', h, cd, ctypes.byref(n))
        t.coarse_dims = tuple(cd)
        t.Vc = _vol(t.coarse_dims)
        t.N = n.value
        return t

    def basis(self):
        B = torch.empty((self.V, self.dof, self.nvec), dtype=torch.complex128, device='cuda')
        _lib.call('qmg_transfer_export', self._h, ctypes.c_void_p(B.data_ptr()), stream_ptr())
        return B

    def _prec(self, t):
        return 'c128' if t.dtype == torch.complex128 else 'c64'

    def prolong(self, uc, out=None):
        """P uc for uc [Vc][N] or [nrhs][Vc][N]."""
        p = self._prec(uc)
        m, cshape = _nrhs(uc, (self.Vc, self.N), 'coarse_in')
        fshape = cshape[:-2] + (self.V, self.dof)
        if out is None:
            out = torch.empty(fshape, dtype=uc.dtype, device=uc.device)
        _lib.call('qmg_prolong', self._h, _dev_ptr(uc, _CDTYPE[p], cshape, 'coarse_in'),
                  _dev_ptr(out, _CDTYPE[p], fshape, 'fine_out'), m, PREC[p], stream_ptr())
        return out

    def restrict(self, f, out=None):
        """R f for f [V][dof] or [nrhs][V][dof]."""
        p = self._prec(f)
        m, fshape = _nrhs(f, (self.V, self.dof), 'fine_in')
        cshape = fshape[:-2] + (self.Vc, self.N)
        if out is None:
            out = torch.empty(cshape, dtype=f.dtype, device=f.device)
        _lib.call('qmg_restrict', self._h, _dev_ptr(f, _CDTYPE[p], fshape, 'fine_in'),
                  _dev_ptr(out, _CDTYPE[p], cshape, 'coarse_out'), m, PREC[p], stream_ptr())
        return out

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None and not getattr(self, '_borrowed', False):
            _lib._lib.qmg_transfer_destroy(h)
            self._h = None


def build_coarse_op(transfer, fine=None, parent=None, storage='c128'):
    """Galerkin product P^+ M P as a new CoarseOp (qmg_build_coarse_op)."""
    h = ctypes.c_void_p()
    _lib.call('qmg_build_coarse_op', transfer._h, fine._h if fine is not None else None,
              parent._h if parent is not None else None, PREC[storage], stream_ptr(), ctypes.byref(h))
    return CoarseOp(transfer.coarse_dims, None, None, storage, _handle=h, _N=transfer.N)


class _BorrowedTransfer(Transfer):
    def __init__(self, handle, fine_dims, dof, nvec, storage):
        self._borrowed = True
        self._h = handle
        self.fine_dims = tuple(fine_dims)
        self.V = _vol(self.fine_dims)
        self.dof, self.nvec, self.storage = dof, nvec, storage
        cd = _lib.c_dims()
        n = ctypes.c_int()
        _lib.call('qmg_transfer_coarse_dims', handle, cd, ctypes.byref(n))
        self.coarse_dims = tuple(cd)
        self.Vc = _vol(self.coarse_dims)
        self.N = n.value


class BiCGStab:
    """Mixed-precision BiCGStab with FP64 reliable updates (qmg_bicgstab_create):
    hi is a complex128 FineOp, lo a FineOp of the same operator in the
    iteration's storage; evenodd selects the red-black (Schur) system."""

    def __init__(self, hi, lo, evenodd=True):
        self.V = hi.V
        self._ops = (hi, lo)
        h = ctypes.c_void_p()
        _lib.call('qmg_bicgstab_create', hi._h, lo._h, int(bool(evenodd)), stream_ptr(), ctypes.byref(h))
        self._h = h

    def solve(self, b, x=None, tol=1e-10, maxit=20000, delta=0.1, check=True):
        if x is None:
            x = torch.empty_like(b)
        p = _lib.BicgstabParams(tol=float(tol), maxit=int(maxit), delta=float(delta))
        info = _lib.SolveInfo()
        st = _lib.lib().qmg_bicgstab_solve(self._h, _dev_ptr(b, torch.complex128, (self.V, 4, 3), 'b'),
                                           _dev_ptr(x, torch.complex128, (self.V, 4, 3), 'x'), ctypes.byref(p),
                                           ctypes.byref(info), stream_ptr())
        out = {'iters': info.outer_iters, 'reliable_updates': info.restarts, 'converged': bool(info.converged),
               'true_rel_residual': info.true_rel_residual, 'seconds': info.seconds, 'status': st}
        if check:
            _lib.check(st, 'qmg_bicgstab_solve')
        return x, out

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.qmg_bicgstab_destroy(h)
            self._h = None


class Multigrid:
    """Adaptive multigrid hierarchy + K-cycle FGCR solver (qmg_mg_create / qmg_mg_gcr_solve).

    levels: list of dicts with keys block, nvec, setup_iters, smoother_steps,
    coarse_tol, coarse_maxit and optionally coarse_storage ('h16' / 'b16': the
    next level's operator in 16-bit storage during the solve), transfer_storage
    ('h16': the level's transfer basis as FP16 pairs in the solve) and, on the last
    entry, coarse_direct (exact coarsest solve by a dense inverse), one per
    coarsened level; starts: list of device complex128 tensors
    [nvec_l][V_l][dof_l]; fine_storage: None or 'h16' / 'b16' for the fine
    operator inside the K-cycle."""

    def __init__(self, dims, gauge, m0, csw, levels, starts, antiperiodic_t=True, inner='c64', fine_storage=None,
                 bases=None):
        """bases (instead of starts): the levels' FP64 transfer bases, complex128
        [V_l][dof_l][nvec_l], as a checkpoint holds them (qmg_mg_create_from_bases)."""
        self.dims = tuple(int(d) for d in dims)
        self.V = _vol(self.dims)
        self.inner = inner
        self.nlevels = len(levels) + 1
        self._cfg = dict(dims=list(self.dims), m0=float(m0), csw=float(csw), antiperiodic_t=bool(antiperiodic_t),
                         inner=inner, fine_storage=fine_storage,
                         levels=[{k: (list(v) if isinstance(v, (tuple, list)) else v) for k, v in L.items()}
                                 for L in levels])
        self._gauge = gauge
        lp = (_lib.LevelParams * max(1, len(levels)))()
        for i, L in enumerate(levels):
            lp[i].block = (ctypes.c_int * 4)(*L['block'])
            lp[i].nvec = int(L['nvec'])
            lp[i].setup_iters = int(L.get('setup_iters', 100))
            lp[i].smoother_steps = int(L.get('smoother_steps', 4))
            lp[i].coarse_tol = float(L.get('coarse_tol', 0.25))
            lp[i].coarse_maxit = int(L.get('coarse_maxit', 10))
            lp[i].coarse_storage = PREC[L['coarse_storage']] if L.get('coarse_storage') else 0
            lp[i].coarse_direct = int(bool(L.get('coarse_direct', False)))
            lp[i].transfer_storage = PREC[L['transfer_storage']] if L.get('transfer_storage') else 0
        vecs, what = (starts, 'starts') if bases is None else (bases, 'bases')
        ptrs = (ctypes.c_void_p * max(1, len(vecs)))()
        for i, t in enumerate(vecs):
            if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
                raise TypeError('%s[%d] must be a contiguous complex128 device tensor' % (what, i))
            ptrs[i] = t.data_ptr()
        self._starts = vecs
        h = ctypes.c_void_p()
        _lib.call('qmg_mg_create' if bases is None else 'qmg_mg_create_from_bases', _lib.c_dims(*self.dims),
                  _dev_ptr(gauge, torch.complex128, (4, self.V, 3, 3), 'gauge'),
                  float(m0), float(csw), int(bool(antiperiodic_t)), self.nlevels, lp, ptrs, PREC[inner],
                  PREC[fine_storage] if fine_storage else 0, stream_ptr(), ctypes.byref(h))
        self._h = h
        self._levels = levels

    def solve(self, b, x=None, tol=1e-10, maxit=500, check=True):
        if x is None:
            x = torch.empty_like(b)
        sp = _lib.SolveParams(tol=float(tol), restart=10, maxit=int(maxit))
        info = _lib.SolveInfo()
        st = _lib.lib().qmg_mg_gcr_solve(self._h, _dev_ptr(b, torch.complex128, (self.V, 4, 3), 'b'),
                                         _dev_ptr(x, torch.complex128, (self.V, 4, 3), 'x'),
                                         ctypes.byref(sp), ctypes.byref(info), stream_ptr())
        out = self._info(info, st)
        if check:
            _lib.check(st, 'qmg_mg_gcr_solve')
        return x, out

    def solve_multi(self, b, x=None, tol=1e-10, maxit=500, check=True):
        """Solve for the right-hand sides b [nrhs][V][4][3] together (qmg_mg_gcr_solve_multi);
        returns x and one info dict per right-hand side."""
        nrhs = int(b.shape[0])
        if x is None:
            x = torch.empty_like(b)
        sp = _lib.SolveParams(tol=float(tol), restart=10, maxit=int(maxit))
        infos = (_lib.SolveInfo * nrhs)()
        st = _lib.lib().qmg_mg_gcr_solve_multi(self._h, _dev_ptr(b, torch.complex128, (nrhs, self.V, 4, 3), 'b'),
                                               _dev_ptr(x, torch.complex128, (nrhs, self.V, 4, 3), 'x'), nrhs,
                                               ctypes.byref(sp), infos, stream_ptr())
        out = [self._info(infos[k], st) for k in range(nrhs)]
        if check:
            _lib.check(st, 'qmg_mg_gcr_solve_multi')
        return x, out

    def _info(self, info, st):
        return {'outer_iters': info.outer_iters, 'level_iters': list(info.level_iters)[:self.nlevels],
                'restarts': info.restarts, 'converged': bool(info.converged),
                'true_rel_residual': info.true_rel_residual, 'seconds': info.seconds,
                'smoother_fallbacks': info.smoother_fallbacks, 'level_seconds': list(info.level_seconds)[:self.nlevels],
                'status': st}

    def solve_record(self, b, maxrec, tol=1e-10, maxit=500):
        """Solve and keep the outer iterates x_1..x_n (complex128 [n][V][4][3])."""
        x = torch.empty_like(b)
        hist = torch.empty((maxrec, self.V, 4, 3), dtype=torch.complex128, device=b.device)
        sp = _lib.SolveParams(tol=float(tol), restart=10, maxit=int(maxit))
        info = _lib.SolveInfo()
        n = ctypes.c_int()
        st = _lib.lib().qmg_mg_gcr_solve_record(self._h, _dev_ptr(b, torch.complex128, (self.V, 4, 3), 'b'),
                                                _dev_ptr(x, torch.complex128, (self.V, 4, 3), 'x'),
                                                ctypes.byref(sp), ctypes.byref(info),
                                                ctypes.c_void_p(hist.data_ptr()), int(maxrec), ctypes.byref(n),
                                                stream_ptr())
        _lib.check(st, 'qmg_mg_gcr_solve_record')
        return x, hist[:n.value], self._info(info, st)

    def solve_record_smoother(self, b, maxrec, tol=1e-10, maxit=500):
        """Solve and keep the level-0 smoother inputs (complex64 [n][V][4][3])."""
        x = torch.empty_like(b)
        hist = torch.empty((maxrec, self.V, 4, 3), dtype=torch.complex64, device=b.device)
        sp = _lib.SolveParams(tol=float(tol), restart=10, maxit=int(maxit))
        info = _lib.SolveInfo()
        n = ctypes.c_int()
        st = _lib.lib().qmg_mg_gcr_solve_record_smoother(
            self._h, _dev_ptr(b, torch.complex128, (self.V, 4, 3), 'b'),
            _dev_ptr(x, torch.complex128, (self.V, 4, 3), 'x'), ctypes.byref(sp), ctypes.byref(info),
            ctypes.c_void_p(hist.data_ptr()), int(maxrec), ctypes.byref(n), stream_ptr())
        _lib.check(st, 'qmg_mg_gcr_solve_record_smoother')
        return x, hist[:n.value], self._info(info, st)

    def make_pairs(self, xstar, hist):
        """(r_k, e_k) = (M (x* - x_k), x* - x_k) as complex64 [n][V][4][3] each."""
        n = hist.shape[0]
        r = torch.empty((n, self.V, 4, 3), dtype=torch.complex64, device=xstar.device)
        e = torch.empty_like(r)
        _lib.call('qmg_mg_make_pairs', self._h, _dev_ptr(xstar, torch.complex128, (self.V, 4, 3), 'xstar'),
                  _dev_ptr(hist, torch.complex128, (n, self.V, 4, 3), 'hist'), int(n),
                  ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(e.data_ptr()), stream_ptr())
        return r, e

    def set_smoother(self, net, mr_steps=0):
        """Learned level-0 smoother (None: MR); mr_steps MR steps follow each accepted network step."""
        _lib.call('qmg_mg_set_smoother', self._h, net._h if net is not None else None)
        _lib.call('qmg_mg_set_smoother_mr_steps', self._h, int(mr_steps))
        self._smoother = net

    def set_evenodd(self, on=True):
        """Red-black preconditioning on every level (qmg_mg_set_evenodd)."""
        _lib.call('qmg_mg_set_evenodd', self._h, int(bool(on)), stream_ptr())

    def set_fine_links(self, link_reals):
        """Links of the K-cycle's fine operator stored with 18 or 12 reals (qmg_mg_set_fine_links)."""
        _lib.call('qmg_mg_set_fine_links', self._h, int(link_reals), stream_ptr())

    def set_level_timing(self, on=True):
        """Per-level device time in the solve info's level_seconds (qmg_mg_set_level_timing)."""
        _lib.call('qmg_mg_set_level_timing', self._h, int(bool(on)))

    def set_smoother_vectors(self, storage=None):
        """Level-0 MR smoother vectors in the red-black form: None (inner precision) or 'h16'
        (qmg_mg_set_smoother_vectors)."""
        _lib.call('qmg_mg_set_smoother_vectors', self._h, PREC[storage] if storage else 0, stream_ptr())

    def set_sap(self, block=(4, 4, 4, 4), iters=4):
        """Level-0 Schwarz (SAP) smoother with `iters` MR steps per block; iters=0 returns to MR."""
        _lib.call('qmg_mg_set_sap', self._h, _lib.c_dims(*block), int(iters), stream_ptr())

    def level(self, l):
        d = _lib.c_dims()
        dof = ctypes.c_int()
        op, T = ctypes.c_void_p(), ctypes.c_void_p()
        _lib.call('qmg_mg_level', self._h, int(l), d, ctypes.byref(dof), ctypes.byref(op), ctypes.byref(T))
        dims = tuple(d)
        cop = None
        if op.value:
            cop = CoarseOp(dims, None, None, self.inner, _handle=op, _N=dof.value)
            cop._borrowed = True
        tr = None
        if T.value:
            tr = _BorrowedTransfer(T, dims, dof.value, int(self._levels[l]['nvec']), self.inner)
        return dims, dof.value, cop, tr

    def save(self, path):
        """Checkpoint the hierarchy to an .npz file: the gauge field, the operator and
        level parameters, and every level's FP64 transfer basis (qmg_transfer_export).
        Multigrid.load rebuilds it without the near-null relaxation, with coarse
        operators bit for bit equal; solver settings made with set_* are not saved."""
        arrays = {'meta': np.frombuffer(json.dumps(self._cfg).encode(), dtype=np.uint8),
                  'gauge': self._gauge.detach().cpu().numpy()}
        for l in range(self.nlevels - 1):
            arrays['basis%d' % l] = self.level(l)[3].basis().cpu().numpy()
        # the autotuner's launch choices fix the stencils' summation order: keep them
        # so that a resumed hierarchy in another process solves bit for bit alike
        import tempfile
        with tempfile.TemporaryDirectory() as d:
            f = os.path.join(d, 'tune.txt')
            tune_cache_save(f)
            with open(f, 'rb') as fh:
                arrays['tune'] = np.frombuffer(fh.read(), dtype=np.uint8)
        np.savez(path, **arrays)

    @classmethod
    def load(cls, path):
        """Resume a hierarchy written by save() (qmg_mg_create_from_bases).  The saved
        launch choices enter the autotuner's cache first when the file was written on
        this device architecture and runtime; otherwise the stencils are tuned anew."""
        with np.load(path, allow_pickle=False) as z:
            c = json.loads(bytes(z['meta']).decode())
            gauge = torch.from_numpy(z['gauge']).to('cuda')
            bases = [torch.from_numpy(z['basis%d' % l]).to('cuda') for l in range(len(c['levels']))]
            tune = bytes(z['tune']) if 'tune' in z.files else b''
        if tune:
            import tempfile
            with tempfile.TemporaryDirectory() as d:
                f = os.path.join(d, 'tune.txt')
                with open(f, 'wb') as fh:
                    fh.write(tune)
                try:
                    tune_cache_load(f)
                except QmgError:
                    pass  # written on another device or runtime: the stencils are tuned anew
        return cls(c['dims'], gauge, c['m0'], c['csw'], c['levels'], None, antiperiodic_t=c['antiperiodic_t'],
                   inner=c['inner'], fine_storage=c['fine_storage'], bases=bases)

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.qmg_mg_destroy(h)
            self._h = None


def quantize_sites(v, prec='h16'):
    """complex64 [V][N] -> (int32 [V][N] packed 16-bit pairs, float32 [V] per-site scales)."""
    V, N = v.shape
    q = torch.empty((V, N), dtype=torch.int32, device=v.device)
    sc = torch.empty((V,), dtype=torch.float32, device=v.device)
    _lib.call('qmg_quantize_sites', _dev_ptr(v, torch.complex64, (V, N), 'in'), ctypes.c_void_p(q.data_ptr()),
              ctypes.c_void_p(sc.data_ptr()), V, N, PREC[prec], stream_ptr())
    return q, sc


def dequantize_sites(q, sc, prec='h16'):
    V, N = q.shape
    out = torch.empty((V, N), dtype=torch.complex64, device=q.device)
    _lib.call('qmg_dequantize_sites', _dev_ptr(q, torch.int32, (V, N), 'in'),
              _dev_ptr(sc, torch.float32, (V,), 'scale'), ctypes.c_void_p(out.data_ptr()), V, N, PREC[prec],
              stream_ptr())
    return out


class PTC:
    """Learned parallel-transport convolution smoother (qmg_ptc_*).  `fine` must be a
    complex64-storage FineOp on the same lattice; it is kept alive by this object."""

    def __init__(self, fine, hidden=8):
        if fine.storage != 'c64':
            raise ValueError('PTC needs a complex64 FineOp')
        self.fine = fine
        self.C = int(hidden)
        self.V = fine.V
        h = ctypes.c_void_p()
        _lib.call('qmg_ptc_create', fine._h, self.C, stream_ptr(), ctypes.byref(h))
        self._h = h

    def wshapes(self):
        return (9, self.C, 1, 4, 4), (9, 1, self.C, 4, 4)

    def set_weights(self, W1, W2):
        s1, s2 = self.wshapes()
        _lib.call('qmg_ptc_set_weights', self._h, _dev_ptr(W1, torch.complex64, s1, 'W1'),
                  _dev_ptr(W2, torch.complex64, s2, 'W2'), stream_ptr())

    def weights(self):
        s1, s2 = self.wshapes()
        W1 = torch.empty(s1, dtype=torch.complex64, device='cuda')
        W2 = torch.empty(s2, dtype=torch.complex64, device='cuda')
        _lib.call('qmg_ptc_get_weights', self._h, ctypes.c_void_p(W1.data_ptr()), ctypes.c_void_p(W2.data_ptr()),
                  stream_ptr())
        return W1, W2

    def forward(self, r, y=None):
        if y is None:
            y = torch.empty_like(r)
        _lib.call('qmg_ptc_forward', self._h, _dev_ptr(r, torch.complex64, (self.V, 4, 3), 'r'),
                  _dev_ptr(y, torch.complex64, (self.V, 4, 3), 'y'), stream_ptr())
        return y

    def zero_grad(self):
        _lib.call('qmg_ptc_zero_grad', self._h, stream_ptr())

    def accumulate(self, r, e):
        _lib.call('qmg_ptc_accumulate_grad', self._h, _dev_ptr(r, torch.complex64, (self.V, 4, 3), 'r'),
                  _dev_ptr(e, torch.complex64, (self.V, 4, 3), 'e'), stream_ptr())

    def accumulate_residual(self, r):
        _lib.call('qmg_ptc_accumulate_grad_residual', self._h, _dev_ptr(r, torch.complex64, (self.V, 4, 3), 'r'),
                  stream_ptr())

    def grad(self):
        s1, s2 = self.wshapes()
        G1 = torch.empty(s1, dtype=torch.complex64, device='cuda')
        G2 = torch.empty(s2, dtype=torch.complex64, device='cuda')
        loss = ctypes.c_double()
        _lib.call('qmg_ptc_get_grad', self._h, ctypes.c_void_p(G1.data_ptr()), ctypes.c_void_p(G2.data_ptr()),
                  ctypes.byref(loss), stream_ptr())
        return G1, G2, loss.value

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _lib.call('qmg_ptc_adam_step', self._h, float(lr), float(beta1), float(beta2), float(eps), stream_ptr())

    def adam_state(self):
        """(m1, v1, m2, v2, steps) (qmg_ptc_get_adam): the Adam moments as complex64 tensors
        shaped like the weights (real and imaginary parts: the moments of the two real
        parameters) and the number of Adam steps taken."""
        s1, s2 = self.wshapes()
        m1, v1 = (torch.empty(s1, dtype=torch.complex64, device='cuda') for _ in range(2))
        m2, v2 = (torch.empty(s2, dtype=torch.complex64, device='cuda') for _ in range(2))
        n = ctypes.c_int()
        _lib.call('qmg_ptc_get_adam', self._h, *(ctypes.c_void_p(t.data_ptr()) for t in (m1, v1, m2, v2)),
                  ctypes.byref(n), stream_ptr())
        return m1, v1, m2, v2, n.value

    def set_adam_state(self, m1, v1, m2, v2, steps):
        s1, s2 = self.wshapes()
        _lib.call('qmg_ptc_set_adam', self._h, _dev_ptr(m1, torch.complex64, s1, 'm1'),
                  _dev_ptr(v1, torch.complex64, s1, 'v1'), _dev_ptr(m2, torch.complex64, s2, 'm2'),
                  _dev_ptr(v2, torch.complex64, s2, 'v2'), int(steps), stream_ptr())

    def save(self, path):
        """Checkpoint the weights and the Adam state to an .npz file."""
        W1, W2 = self.weights()
        m1, v1, m2, v2, n = self.adam_state()
        np.savez(path, W1=W1.cpu().numpy(), W2=W2.cpu().numpy(), m1=m1.cpu().numpy(), v1=v1.cpu().numpy(),
                 m2=m2.cpu().numpy(), v2=v2.cpu().numpy(), steps=np.array(n, dtype=np.int64))

    def load(self, path):
        """Restore weights and Adam state written by save(); training resumes where it stopped."""
        with np.load(path, allow_pickle=False) as z:
            t = {k: torch.from_numpy(z[k]).to('cuda') for k in ('W1', 'W2', 'm1', 'v1', 'm2', 'v2')}
            n = int(z['steps'])
        self.set_weights(t['W1'], t['W2'])
        self.set_adam_state(t['m1'], t['v1'], t['m2'], t['v2'], n)

    def __del__(self):
        h = getattr(self, '_h', None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.qmg_ptc_destroy(h)
            self._h = None


def apply_mrhs_multi(ops, u16s, uscales, outs, grid=0):
    """One persistent launch of the multi-RHS operator over several coarse operators
    (qmg_coarse_dslash_mrhs_multi); u16s/uscales/outs as for CoarseOp.apply_mrhs."""
    n = len(ops)
    nrhs = int(u16s[0].shape[1])
    P = ctypes.c_void_p * n
    for op, u, sc, o in zip(ops, u16s, uscales, outs):
        _dev_ptr(u, torch.int32, (op.V, nrhs, op.N), 'in')
        _dev_ptr(sc, torch.float32, (op.V, nrhs), 'in_scale')
        _dev_ptr(o, torch.complex64, (op.V, nrhs, op.N), 'out')
    _lib.call('qmg_coarse_dslash_mrhs_multi', n, P(*[op._h.value for op in ops]), P(*[u.data_ptr() for u in u16s]),
              P(*[s.data_ptr() for s in uscales]), P(*[o.data_ptr() for o in outs]), nrhs, int(grid), stream_ptr())
    return outs

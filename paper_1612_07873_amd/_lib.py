"""ctypes declarations of the qmg C ABI (include/qmg.h).  Marshalling only."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, 'libqmg.so')

c_int, c_double, c_void_p, c_char_p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p
c_int_p = ctypes.POINTER(ctypes.c_int)
c_dims = ctypes.c_int * 4

QMG_C128, QMG_C64, QMG_H16, QMG_B16 = 0, 1, 2, 3
PREC = {'c128': QMG_C128, 'c64': QMG_C64, 'h16': QMG_H16, 'b16': QMG_B16}
STATUS = {0: 'QMG_OK', 1: 'QMG_ERR_ARG', 2: 'QMG_ERR_SHAPE', 3: 'QMG_ERR_PREC', 4: 'QMG_ERR_HIP',
          5: 'QMG_ERR_NOMEM', 6: 'QMG_ERR_NOCONV', 7: 'QMG_ERR_NONFINITE', 8: 'QMG_ERR_STATE'}

# name -> (restype, argtypes)
SIGNATURES = {
    'qmg_last_error': (c_char_p, []),
    'qmg_version': (c_int, []),
    'qmg_sync': (c_int, [c_void_p]),
    'qmg_stream_read': (c_int, [c_void_p, ctypes.c_longlong, c_void_p, c_int, c_void_p]),
    'qmg_coarse_op_create': (c_int, [c_dims, c_int, c_void_p, c_void_p, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_coarse_op_export': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    'qmg_coarse_dslash': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_coarse_dslash_mrhs_c64': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_coarse_op_set_launch': (c_int, [c_void_p, c_int, c_int]),
    'qmg_coarse_op_get_prefetch': (c_int, [c_void_p, c_int_p]),
    'qmg_coarse_op_tune': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p,
                                   ctypes.POINTER(ctypes.c_float)]),
    'qmg_coarse_op_tune_mrhs': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p,
                                        ctypes.POINTER(ctypes.c_float)]),
    'qmg_tune_cache_save': (c_int, [c_char_p, c_int_p]),
    'qmg_tune_cache_load': (c_int, [c_char_p, c_int_p]),
    'qmg_tune_cache_clear': (c_int, []),
    'qmg_coarse_dslash_mrhs': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_coarse_op_set_mrhs_tiles': (c_int, [c_void_p, c_int, c_int]),
    'qmg_coarse_op_get_mrhs_tiles': (c_int, [c_void_p, c_int, c_int_p]),
    'qmg_coarse_dslash_mrhs_multi': (c_int, [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p),
                                             ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int, c_int, c_void_p]),
    'qmg_coarse_dslash_scaled': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_quantize_sites': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_longlong, c_int, c_int, c_void_p]),
    'qmg_dequantize_sites': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_longlong, c_int, c_int, c_void_p]),
    'qmg_coarse_op_get_launch': (c_int, [c_void_p, c_int_p, c_int_p]),
    'qmg_coarse_op_destroy': (None, [c_void_p]),
    'qmg_fine_op_create': (c_int, [c_dims, c_void_p, c_double, c_double, c_int, c_int, c_void_p,
                                   ctypes.POINTER(c_void_p)]),
    'qmg_wilson_clover_dslash': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_wilson_clover_dslash_scaled': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_fine_op_export_clover': (c_int, [c_void_p, c_void_p, c_void_p]),
    'qmg_fine_op_export_links': (c_int, [c_void_p, c_void_p, c_void_p]),
    'qmg_fine_op_destroy': (None, [c_void_p]),
    'qmg_transfer_create': (c_int, [c_dims, c_int, c_dims, c_int, c_void_p, c_int, c_void_p,
                                    ctypes.POINTER(c_void_p)]),
    'qmg_transfer_coarse_dims': (c_int, [c_void_p, c_int_p, c_int_p]),
    'qmg_transfer_export': (c_int, [c_void_p, c_void_p, c_void_p]),
    'qmg_wilson_clover_schur_scaled': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_mg_set_smoother_vectors': (c_int, [c_void_p, c_int, c_void_p]),
    'qmg_transfer_import': (c_int, [c_dims, c_int, c_dims, c_int, c_void_p, c_int, c_void_p,
                                    ctypes.POINTER(c_void_p)]),
    'qmg_prolong': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_restrict': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_transfer_destroy': (None, [c_void_p]),
    'qmg_build_coarse_op': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_wilson_clover_schur': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_wilson_clover_schur_source': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_wilson_clover_schur_reconstruct': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_wilson_clover_schur_noalloc': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_coarse_op_prepare_schur': (c_int, [c_void_p, c_void_p]),
    'qmg_fine_op_create_ex': (c_int, [c_dims, c_void_p, c_double, c_double, c_int, c_int, c_int, c_void_p,
                                      ctypes.POINTER(c_void_p)]),
    'qmg_wilson_clover_sap': (c_int, [c_void_p, c_dims, c_int, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_coarse_dslash_schur': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_coarse_schur_source': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
    'qmg_coarse_schur_reconstruct': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int, c_void_p]),
}



class LevelParams(ctypes.Structure):
    _fields_ = [('block', c_int * 4), ('nvec', c_int), ('setup_iters', c_int), ('smoother_steps', c_int),
                ('coarse_tol', c_double), ('coarse_maxit', c_int), ('coarse_storage', c_int),
                ('coarse_direct', c_int), ('transfer_storage', c_int)]


class SolveParams(ctypes.Structure):
    _fields_ = [('tol', c_double), ('restart', c_int), ('maxit', c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [('outer_iters', c_int), ('level_iters', c_int * 4), ('restarts', c_int), ('converged', c_int),
                ('true_rel_residual', c_double), ('seconds', c_double), ('smoother_fallbacks', c_int),
                ('level_seconds', c_double * 4)]


class BicgstabParams(ctypes.Structure):
    _fields_ = [('tol', c_double), ('maxit', c_int), ('delta', c_double)]


SIGNATURES.update({
    'qmg_bicgstab_create': (c_int, [c_void_p, c_void_p, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_bicgstab_solve': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(BicgstabParams),
                                   ctypes.POINTER(SolveInfo), c_void_p]),
    'qmg_bicgstab_destroy': (None, [c_void_p]),
    'qmg_mg_create': (c_int, [c_dims, c_void_p, c_double, c_double, c_int, c_int, ctypes.POINTER(LevelParams),
                              ctypes.POINTER(c_void_p), c_int, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_mg_create_from_bases': (c_int, [c_dims, c_void_p, c_double, c_double, c_int, c_int,
                                         ctypes.POINTER(LevelParams), ctypes.POINTER(c_void_p), c_int, c_int,
                                         c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_mg_gcr_solve': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveParams),
                                 ctypes.POINTER(SolveInfo), c_void_p]),
    'qmg_mg_gcr_solve_record_smoother': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveParams),
                                                 ctypes.POINTER(SolveInfo), c_void_p, c_int, c_int_p, c_void_p]),
    'qmg_mg_gcr_solve_multi': (c_int, [c_void_p, c_void_p, c_void_p, c_int, ctypes.POINTER(SolveParams),
                                       ctypes.POINTER(SolveInfo), c_void_p]),
    'qmg_mg_level': (c_int, [c_void_p, c_int, c_int_p, c_int_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p)]),
    'qmg_mg_fine_op': (c_int, [c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_mg_destroy': (None, [c_void_p]),
    'qmg_mg_set_smoother': (c_int, [c_void_p, c_void_p]),
    'qmg_mg_set_evenodd': (c_int, [c_void_p, c_int, c_void_p]),
    'qmg_mg_set_fine_links': (c_int, [c_void_p, c_int, c_void_p]),
    'qmg_mg_set_level_timing': (c_int, [c_void_p, c_int]),
    'qmg_mg_set_sap': (c_int, [c_void_p, c_dims, c_int, c_void_p]),
    'qmg_mg_set_smoother_mr_steps': (c_int, [c_void_p, c_int]),
    'qmg_mg_gcr_solve_record': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(SolveParams),
                                        ctypes.POINTER(SolveInfo), c_void_p, c_int, c_int_p, c_void_p]),
    'qmg_mg_make_pairs': (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_create': (c_int, [c_void_p, c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    'qmg_ptc_set_weights': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_get_weights': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_get_adam': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int_p, c_void_p]),
    'qmg_ptc_set_adam': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    'qmg_ptc_forward': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_accumulate_grad': (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_zero_grad': (c_int, [c_void_p, c_void_p]),
    'qmg_ptc_accumulate_grad_residual': (c_int, [c_void_p, c_void_p, c_void_p]),
    'qmg_ptc_get_grad': (c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p]),
    'qmg_ptc_adam_step': (c_int, [c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p]),
    'qmg_ptc_destroy': (None, [c_void_p]),
})

_lib = None


class QmgError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__('%s: %s (%s)' % (where, msg, STATUS.get(status, status)))
        self.status = status


def lib():
    """Load libqmg.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError('libqmg.so is not built (%s); run python -m paper_1612_07873_amd.build'
                               % LIB_PATH)
        l = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def check(status, where):
    if status != 0:
        msg = lib().qmg_last_error()
        raise QmgError(status, where, msg.decode() if msg else '')


def call(name, *args):
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st

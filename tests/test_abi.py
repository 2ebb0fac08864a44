"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, 'include', '*.h')):
        text = open(h).read()
        text = re.sub(r'/\*.*?\*/', '', text, flags=re.S)
        names |= set(re.findall(r'\b(qmg_[a-z0-9_]+)\s*\(', text))
    return sorted(names)


@pytest.fixture(scope='module')
def lib():
    from paper_1612_07873_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail('libqmg.so missing: build it with python -m paper_1612_07873_amd.build')
    return _lib.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 8
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_header_function():
    from paper_1612_07873_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_version_and_empty_error(lib):
    assert lib.qmg_version() >= 100


def test_coarse_create_rejects_bad_arguments_without_a_device(lib):
    from paper_1612_07873_amd import _lib
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    cases = [((2, 2, 1, 2), 48, _lib.QMG_C128, _lib.QMG_ERR_SHAPE if hasattr(_lib, 'QMG_ERR_SHAPE') else 2),
             ((2, 2, 2, 2), 47, _lib.QMG_C128, 2),
             ((2, 2, 2, 2), 0, _lib.QMG_C128, 2),
             ((2, 2, 2, 2), 130, _lib.QMG_C128, 2),
             ((2, 2, 2, 2), 48, 7, 3)]
    for dims, N, prec, want in cases:
        st = lib.qmg_coarse_op_create(_lib.c_dims(*dims), N, fake, fake, prec, None, ctypes.byref(h))
        assert st == want, (dims, N, prec, st)
        assert lib.qmg_last_error()
        assert not h.value
    st = lib.qmg_coarse_op_create(_lib.c_dims(2, 2, 2, 2), 48, None, fake, 0, None, ctypes.byref(h))
    assert st == 1
    st = lib.qmg_coarse_dslash(None, fake, fake, 1, 0, None)
    assert st == 1
    # a right-hand-side count out of range is refused before anything is touched
    for name in ('qmg_coarse_dslash', 'qmg_wilson_clover_dslash', 'qmg_prolong', 'qmg_restrict'):
        for nrhs in (0, -3, 1025):
            st = getattr(lib, name)(fake, fake, ctypes.c_void_p(8), nrhs, 0, None)
            assert st == 1, (name, nrhs, st)
            assert b'nrhs' in lib.qmg_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libqmg.so the binding raises; there is no CPU fallback."""
    from paper_1612_07873_amd import _lib
    monkeypatch.setattr(_lib, '_lib', None)
    monkeypatch.setattr(_lib, 'LIB_PATH', str(tmp_path / 'libqmg.so'))
    with pytest.raises(RuntimeError, match='not built'):
        _lib.lib()

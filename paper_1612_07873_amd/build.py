"""Build step: compile every HIP source under csrc/ for gfx950 and link the
C-ABI shared library libqmg.so next to this file.

Run as ``python -m paper_1612_07873_amd.build`` (or through the package's
build entry point).  It always recompiles.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
OUT = os.path.join(HERE, 'libqmg.so')
BUILD_DIR = os.path.join(ROOT, '_build', 'qmg')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
ARCH = 'gfx950'

FLAGS = ['--offload-arch=' + ARCH, '-O3', '-std=c++17', '-fPIC', '-Wall', '-Wno-unused-function',
         # packed FP32 instructions are kept out of all device code
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-I' + os.path.join(ROOT, 'include')]


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + '.o')
    cmd = [HIPCC] + FLAGS + ['-c', src, '-o', obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msg = '\n'.join(l for l in (p.stdout + p.stderr).splitlines()
                    if 'packed-fp32-ops' not in l)
    if p.returncode != 0:
        raise RuntimeError('hipcc failed on %s:\n%s' % (src, msg))
    return obj, msg


def build(verbose=True):
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, '*.hip')))
    if not srcs:
        raise RuntimeError('no HIP sources under %s' % CSRC)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    for obj, msg in results:
        if msg.strip() and verbose:
            print(msg, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = OUT + '.tmp'
    cmd = [HIPCC, '--offload-arch=' + ARCH, '-shared', '-fPIC', '-o', tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError('link failed:\n%s%s' % (p.stdout, p.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print('built %s from %d sources' % (OUT, len(srcs)))
    return OUT


if __name__ == '__main__':
    build()

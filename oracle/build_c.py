"""Build the oracle's C part (oracle/csrc/*.c) into oracle/_oracle_c.so with gcc."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, '_oracle_c.so')


def build(verbose=True):
    srcs = sorted(glob.glob(os.path.join(HERE, 'csrc', '*.c')))
    cmd = ['gcc', '-O2', '-fopenmp', '-fPIC', '-shared', '-std=c11', '-o', OUT + '.tmp'] + srcs + ['-lm']
    subprocess.run(cmd, check=True)
    os.replace(OUT + '.tmp', OUT)
    if verbose:
        print('built %s' % OUT)
    return OUT


if __name__ == '__main__':
    build()

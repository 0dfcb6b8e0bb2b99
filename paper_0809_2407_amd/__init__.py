"""TSQR on AMD Instinct MI355X (gfx950): the communication-avoiding Householder
QR of tall-skinny matrices of Demmel, Grigori, Hoemmen and Langou (arXiv
0809.2407), as hand-written HIP kernels behind a C ABI (include/tsqr.h).

Submodules: ``tsqr`` (the Python binding, needs torch), ``build`` (compiles
libtsqr.so for gfx950)."""

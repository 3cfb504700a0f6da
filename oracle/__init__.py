"""FP64 CPU oracle for the Monte-Carlo Lyman-alpha transport path.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import, call, link or run anything in this
package. It is an independent, plain reimplementation of what the path
computes, written from the paper (arXiv:2312.11448): physics scalars and closed
forms in ``physics``, the packet walk and the resonant-scattering Monte Carlo
in the C file behind ``walker``, brute-force checks in ``brute``, the
recombination histories in ``recombination``, and the features, network, loss
gradient and Adam update of the mixing-correction surrogate in ``surrogate``.
It shares no code with the HIP library and never imports it.

Parity unpinned: none of the functions here is left without a pin. The
values of the paper's mixing-length and escape-against-flow figures are not
printed, so the experiments that reproduce them are checked against the
paper's statements and the closed forms only.
"""
from . import physics, walker, brute, surrogate, recombination  # noqa: F401
from .walker import run_box, Prepared, philox4x32_10, quantize, allocate  # noqa: F401

"""FP64 CPU oracle for the Monte-Carlo Lyman-alpha transport path.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import, call, link or run anything in this
package. It is an independent, plain reimplementation of what the path
computes, written from the paper (arXiv:2312.11448): physics scalars and closed
forms in ``physics``, the packet walk in the C file behind ``walker``,
brute-force checks in ``brute``, and the features, network, loss gradient and
Adam update of the mixing-correction surrogate in ``surrogate``. It shares no code with the HIP library and
never imports it.

Parity unpinned: none of the functions here is left without a pin; the
physical fidelity of the streaming model against the paper's
resonant-scattering Monte Carlo (its mixing-length and escape-vs-flow figures,
whose data are not printed) is not pinned.
"""
from . import physics, walker, brute, surrogate  # noqa: F401
from .walker import run_box, Prepared, philox4x32_10, quantize, allocate  # noqa: F401

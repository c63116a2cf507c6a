"""FP64 CPU oracle for the FastPM-with-neutrinos particle-mesh step.

TEST INFRASTRUCTURE ONLY: this package exists so that the GPU library can be
checked against a plain, slow, obviously correct implementation written from
the paper (Bayer, Banerjee & Feng, arXiv:2007.13394).  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the GPU library and never imports it.
"""
from .orc import *  # noqa: F401,F403

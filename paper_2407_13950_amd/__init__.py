"""MI355X-native multiple-shooting quantum optimal control: the penalty objective
and its discrete-adjoint gradient on hand-written CDNA4 HIP kernels behind a C ABI.

Importing the package loads nothing native; `paper_2407_13950_amd.qoc` loads the
HIP library (and fails loudly when it is missing).
"""
__all__ = ["workloads", "qoc"]

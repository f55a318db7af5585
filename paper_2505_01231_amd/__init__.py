"""MI355X-native polyspectrum estimator (arXiv 2505.01231).

The HIP library (libpolyspec.so) is loaded on first use of ``Plan`` or
``enumerate_combos``; importing this package (e.g. for ``synth``) does not
load it.
"""
import importlib

__all__ = ["Plan", "Spectra", "Graph", "Streamer", "Accumulator", "enumerate_combos", "quasi_spectra", "m_dependence",
           "synth"]


def __getattr__(name):
    if name in ("Plan", "Spectra", "Graph", "Streamer", "Accumulator", "enumerate_combos", "quasi_spectra",
                "m_dependence"):
        return getattr(importlib.import_module(__name__ + ".polyspec"), name)
    if name == "synth":
        return importlib.import_module(__name__ + ".synth")
    raise AttributeError(name)

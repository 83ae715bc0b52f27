"""MI355X-native hot path of NL-RMM-GKS (angle-parameterised parallel-beam CT).

Submodules: ``synth`` (seeded inputs), ``ops`` (C-ABI entry points over torch
tensors), ``build`` (hipcc build of libnlrmm.so).
"""
__all__ = ["synth", "ops", "build"]

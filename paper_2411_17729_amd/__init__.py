"""MI355X-native fast cascade for state-space models (Beylkin, arXiv 2411.17729).

The compute path lives in the HIP library ``libssm_cascade.so`` built from
``csrc/``; ``binding`` marshals arguments for its C entry points and
``cascade`` wraps them for PyTorch tensors. Nothing is imported eagerly so
that the seeded input generators in ``workloads`` load without a GPU stack.
"""

__all__ = ["workloads", "binding", "cascade", "build"]

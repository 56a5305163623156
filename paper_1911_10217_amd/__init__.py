"""HIP (gfx950) implementation of the per-frame hot path of Reinforcement
Lightcuts Learning (Pantaleoni, arXiv:1911.10217) behind the C ABI of
include/rlc.h.

Modules:
  rlc     - Python binding of librlc.so (argument marshalling only)
  scenes  - seeded synthetic input scenes
  build   - compiles librlc.so in-tree with hipcc
"""

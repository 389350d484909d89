"""MI355X (gfx950) domain decomposition for entropic unbalanced optimal transport.

The solver is the HIP library libdd_uot.so behind the C ABI of
include/dd_uot.h; `binding` is its ctypes mirror (same function names) and
`inputs` draws the seeded synthetic marginals.
"""

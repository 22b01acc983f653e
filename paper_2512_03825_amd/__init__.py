"""Parallel-tempering Metropolis sampling of lattice spin models on MI355X (gfx950).

The method (arXiv 2512.03825): Metropolis-Hastings with Parallel Tempering on
Ising-type lattices.  The hot path -- checkerboard sweeps, energy/magnetisation
bookkeeping, replica exchange, records -- runs in hand-written HIP kernels behind
the C ABI of include/pt.h; ``paper_2512_03825_amd.pt`` is its ctypes binding.
"""
__all__ = ["pt", "workloads"]

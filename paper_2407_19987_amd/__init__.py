"""MI355X (gfx950) engine for the HOBO hot path of HOBOTAN (arXiv 2407.19987):
batched energies, single-flip energy changes and batched Metropolis
annealing of higher-order binary optimisation problems, in hand-written HIP
kernels behind the C-ABI of include/hobo.h.

``from paper_2407_19987_amd import hobo`` loads the built library (see
``paper_2407_19987_amd.build``)."""

__all__ = ["hobo"]

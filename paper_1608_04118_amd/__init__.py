"""MI355X-native LTNE MRT lattice Boltzmann step (Liu & He, arXiv:1608.04118)."""

"""MI355X-native real-time TDDFT hot path (arXiv:1912.07921): KS H.psi on a uniform grid, Taylor-4 ETRS propagation, density, LDA exchange and dipole, through a C ABI (libks)."""

"""MI355X-native reversible 3D FDTD hot path (arXiv 2412.12360)."""

"""FP64 CPU oracle of the FDTD hot path.  Test infrastructure only."""

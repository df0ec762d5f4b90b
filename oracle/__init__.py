"""FP64 CPU oracle of the H^2 matrix-vector product. Test infrastructure only."""

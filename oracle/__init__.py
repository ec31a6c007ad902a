"""Plain FP64 CPU oracle of the moving-particle D3Q19 TRT step (test infrastructure only)."""

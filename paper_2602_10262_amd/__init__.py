"""MI355X-native FP8 GEMM (dense and 2:4 structured-sparse) on gfx950."""

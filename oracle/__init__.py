"""CPU FP64 oracle: test infrastructure only (tests, smoke check, CPU-baseline leg of the benchmark)."""

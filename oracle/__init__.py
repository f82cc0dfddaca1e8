"""Plain CPU FP64 oracle of the hot path -- test infrastructure only."""

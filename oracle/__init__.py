"""CPU FP64 oracle (test infrastructure only; see admm.py for the contract)."""

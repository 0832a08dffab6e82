"""Placeholder bench (replaced below once the FMM path is measured)."""

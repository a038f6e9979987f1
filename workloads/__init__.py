"""Seeded synthetic workloads (inputs only)."""

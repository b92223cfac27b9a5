"""Seeded synthetic inputs shared by the oracle tests and the GPU path."""

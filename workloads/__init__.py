"""Seeded synthetic workloads (input generators and frozen config constants).

Holds none of the method's arithmetic; shared by the oracle tests, the GPU
tests and the bench so that both sides score identical inputs.
"""

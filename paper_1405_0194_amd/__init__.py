"""MI355X-native hot path of the PEXSI method (pole expansion + selected
inversion): pole table, symbolic analysis, batched complex-symmetric
supernodal LDL^T, selected inversion, pole sum and inertia counts.

The compiled library (``libpexsi_hip.so``) is loaded lazily by
``paper_1405_0194_amd.binding``; importing this package alone loads nothing.
"""
__all__ = ["api", "binding", "lattice"]

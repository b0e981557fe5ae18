"""MI355X-native implicit gas-kinetic scheme (IGKS) hot path.

Importing the package loads nothing native; ``paper_1709_00803_amd.igks``
holds the binding to the HIP library and ``meshgen`` the synthetic inputs.
"""

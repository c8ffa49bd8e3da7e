"""MI355X-native BSSN right-hand side and RK4 step (Chemora hot path).

``paper_1307_6488_amd.chemora`` is the binding of the HIP library
(``libchemora.so``); ``paper_1307_6488_amd.inputs`` holds the seeded
synthetic grids and initial data.  Importing the package loads nothing.
"""

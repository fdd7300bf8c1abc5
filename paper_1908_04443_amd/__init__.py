"""MI355X-native pseudopotential lattice Boltzmann step with contact-angle
wall schemes on curved (staircase) boundaries.

Importing the package loads nothing; the GPU library is loaded on first use
by :mod:`paper_1908_04443_amd.lbm`.
"""

"""EXACT on MI355X: projected extragradient for single-material polychromatic
CT, with a Joseph projector pair written in HIP for gfx950 behind a C ABI.

Importing the package loads nothing; `paper_2503_19925_amd.exact` binds the
compiled library (and fails loudly if it is missing), `synth` generates
seeded synthetic scans.
"""

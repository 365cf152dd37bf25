"""MI355X-native implementation of the PORTA hot path (arXiv:1307.4217).

Importing the package is cheap: the HIP library is loaded on first use by
`paper_1307_4217_amd.porta`.
"""
__version__ = "0.1.0"

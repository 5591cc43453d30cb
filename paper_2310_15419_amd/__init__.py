"""MI355X-native sketch A_hat = S A (random dense S regenerated on the fly).

The compute path lives in the HIP library built from ``csrc/``; the Python
binding in ``binding.py`` marshals arguments only.  Importing the package does
not load the library; the first call into ``binding`` does, and fails loudly
if it is missing.
"""

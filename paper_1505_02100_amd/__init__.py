"""libkdeplugin: MI355X-native PLUGIN bandwidth selection for Gaussian KDE.

The HIP library and its ctypes binding live in :mod:`paper_1505_02100_amd.kdeplugin`;
importing that module loads ``libkdeplugin.so`` and fails loudly if it is
missing.  :mod:`paper_1505_02100_amd.synth` draws the seeded synthetic samples.
"""
__all__ = ["kdeplugin", "synth"]

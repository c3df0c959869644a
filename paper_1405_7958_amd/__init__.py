"""MI355X-native per-tile nucleus segmentation (hot path of the Region
Templates example application, Sec. 5.1).

The compute path lives in the HIP library ``librtseg.so`` (see ``rtseg.py`` for
the Python binding of its C ABI); ``synth`` draws seeded synthetic tiles.
Nothing is loaded at import time.
"""

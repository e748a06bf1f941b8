"""MI355X-native hot path of time-domain extended-source waveform inversion.

The compute path is the C-ABI library ``libesi.so`` (HIP kernels for gfx950)
reached through :mod:`paper_2211_06300_amd.esi`; importing this package does
not load it, so the input generators in :mod:`paper_2211_06300_amd.inputs` can
be used without a GPU.
"""

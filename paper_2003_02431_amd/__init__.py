"""MI355X-native multigrid solve of the agglomerated cut-cell SIP system of the
extended DG method (HIP kernels for gfx950 behind the C-ABI in include/xdg.h).

The Python side only marshals arguments: see `binding`.  Importing the
binding requires the built library (paper_2003_02431_amd/libxdg.so)."""

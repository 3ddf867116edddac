"""Space-switching BGV hot path on MI355X (gfx950).

Modules:
  bgv    -- ctypes binding of libbgv.so (the C-ABI in include/bgv.h); importing it
            requires the built library and never falls back to another path
  synth  -- seeded synthetic inputs (keys' randomness, encryption randomness, data)
  build  -- hipcc build of libbgv.so
"""

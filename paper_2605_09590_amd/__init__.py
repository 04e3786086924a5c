"""PICO noise maps on AMD Instinct MI355X (gfx950).

The product is the C-ABI library ``libpico.so`` (include/pico.h) built from
``csrc/``; ``paper_2605_09590_amd.pico`` is its Python binding and
``paper_2605_09590_amd.build`` compiles it.
"""

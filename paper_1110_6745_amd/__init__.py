"""okpz: octahedron-model KPZ growth on AMD MI355X (HIP, gfx950).

The product path is the C-ABI library ``libokpz.so`` (declared in
``include/okpz.h``); ``paper_1110_6745_amd.okpz`` binds it.
"""

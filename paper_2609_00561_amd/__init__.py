"""MI355X-native block-multicolored ICCG (IC(0)-preconditioned CG with ABMC or
Leiden block multi-coloring).  The solver lives in libiccg.so (HIP for gfx950
plus host C++); ``iccg`` is its ctypes binding."""
__all__ = ["iccg"]

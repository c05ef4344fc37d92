"""Robust rotation estimation by quaternion-circle voting on MI355X (gfx950).

The compute path is the HIP library ``librotvote.so`` behind the C-ABI in
``include/rotvote.h``; ``rotvote.Solver`` is its thin Python binding.
"""
__all__ = ["datagen", "rotvote", "build"]

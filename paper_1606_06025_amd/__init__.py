"""MI355X-native speculative-greedy graph colouring (Chen et al., Sec. 3).

The colouring runs in the HIP library libcsrcolor.so (C-ABI in include/csrcolor.h);
``api`` marshals torch device tensors and streams into it, ``graphs`` generates
seeded synthetic inputs.
"""
__version__ = "0.1.0"

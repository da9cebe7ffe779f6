"""fastfocus: MI355X-native layered BTTB sensitivity operator (G, G^T via BCCB embedding
and hand-written HIP 2D FFTs) and the GKB / RSVD / IRLS focusing inversion built on it.

The compute path lives in the C-ABI library ``libfastfocus.so`` (HIP for gfx950); the
Python modules only marshal arguments.  Importing this package does not load the
library; the first operator call does, and fails loudly if it is missing.
"""

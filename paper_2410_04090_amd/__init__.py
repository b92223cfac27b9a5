"""MI355X (gfx950) stereo visual-SLAM front-end: pyramid, FAST with Bounded
Rectification, Pyramidal Culling and Aggregation, ORB + rBRIEF and
rectified-row stereo matching, as hand-written HIP kernels behind a C ABI
(include/vsfe.h) with a thin ctypes binding."""
from . import vsfe  # noqa: F401

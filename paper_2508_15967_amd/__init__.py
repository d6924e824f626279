"""raygraph for MI355X: compiled dispersion-relation graphs driving FP64 ray
tracing on gfx950.  The native library is loaded by ``raygraph`` on first
use; ``workloads`` (seeded inputs) imports without it."""

"""MI355X (gfx950) implementation of the time step of the hybrid
pseudopotential phase-change LBM for pool boiling with conjugate heat transfer
(arXiv:1911.10747).  The compute path is the HIP library libpoolboil.so behind
the C ABI of include/poolboil.h; `poolboil` is its ctypes binding, `presets`
builds configurations, `serve` the continuous-batching job server and
`autotune` the tile tuner.  Submodules load lazily so that building does not
need the library to exist yet."""

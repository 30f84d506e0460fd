"""MI355X-native LoD-select + Gaussian-splat path ("A LoD of Gaussians",
arXiv 2507.01110): HIP kernels behind the C ABI of include/lodgs.h.

Submodules: `_lib` (ctypes declarations), `lodgs` (scene, frame, calls),
`autograd` (torch.autograd.Function), `server` (batched render serving),
`build` (compiles liblodgs.so).  Importing the package loads nothing.
"""

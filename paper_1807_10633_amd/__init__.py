"""MI355X (gfx950) hot path of screened orbital-space VMC.

``paper_1807_10633_amd.vmc`` binds the C ABI of ``libvmc.so`` (include/vmc.h);
``paper_1807_10633_amd.autograd`` wraps the gradient-ratio backward as a
``torch.autograd.Function``; ``paper_1807_10633_amd.build`` compiles the library.
Importing the package loads nothing; the first call into ``vmc`` loads the
library and raises if it has not been built.
"""

"""MI355X (gfx950) mixed-precision geometric multigrid + FP64 iterative
refinement for Poisson's equation (Oo & Vogel, arXiv 2007.07539).

``paper_2007_07539_amd.mgir`` binds the C ABI of ``libmgir.so``;
``paper_2007_07539_amd.workloads`` generates the seeded synthetic inputs.
"""

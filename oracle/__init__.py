"""Plain FP64 CPU oracle of the Greedy Frank-Wolfe segmentation method.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU leg of the
benchmark may import it.  It shares no code with the HIP library."""

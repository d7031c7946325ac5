"""MI355X-native task-DAG executor (Yadav et al., "On the Duality of Task and
Actor Programming Models"): the compiled-graph execution of Algorithm 1 as
persistent HIP kernels for gfx950, behind the C ABI in include/taskgraph.h."""

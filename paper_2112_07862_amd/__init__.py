"""MI355X (gfx950) manifold-graph embedding: the disconnected two-hop
difference matrix Q, eps = lambda_2(Q), mu, the degree-equalising B and the
first K generalized eigenvectors of (A = L - mu Q + eps I, B) by LOBPCG, all
in hand-written HIP kernels behind the C ABI of include/membed.h."""
from ._lib import LIB_PATH, load  # noqa: F401
from .api import (  # noqa: F401
    DeviceCSR, GraphOps, MembedError, Server, betweenness, betweenness_workspace_bytes,
    build_graph_ops, build_workspace_bytes, cluster_scores, cluster_workspace_bytes, embed,
    embed_batch, embed_batch_workspace_bytes, gmm, kernel_timing, kernel_timing_read, kmeans,
    knn_graph, knn_workspace_bytes, make_opts,
    server_request_bytes, step_form, step_form_reset, to_device,
)

"""FP64 CPU oracle of the relational layer.  Test infrastructure only: the
HIP library never imports it (see relnn_oracle's header)."""

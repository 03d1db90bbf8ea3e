"""MI355X-native batched limit-order-book environment step (JaxMARL-HFT hot path)."""

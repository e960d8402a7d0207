"""MI355X-native k-register Gumbel-Max sketch (FastGM and plain forms)."""
